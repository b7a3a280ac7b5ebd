// The W-tensor form of the recursion (Sec. 3, Eqs. 3.3-3.4), with the propagator 1/K^2 that
// the printed Eq. 3.3 leaves implicit:
//   J[m..n]     = 1/K^2 sum_i [ W[i+1..n] . J[m..i] - W[m..i] . J[i+1..n] ],
//   W[m..n]_mu,nu = 2 J_mu K_nu - K_mu J_nu + sum_i ( J_mu[m..i] J_nu[i+1..n] - J_mu[i+1..n] J_nu[m..i] ),
// (W . J)_mu = sum_nu W_mu,nu g_nu,nu J^nu.  It undoes the double sum of the four-gluon terms
// (O(n^3) instead of O(n^4) work) at the price of a 4x4 complex tensor per span.
//
// On the device one event takes 16 lanes: lane (mu, nu) = (l / 4, l % 4) of the group holds
// W_mu,nu of every span in registers and the mu-component of every current; a current's
// components are published in LDS (one 16-lane group per event, 4 events per wave), so that
// lane (mu, nu) reads J_nu there.  (W . J)_mu is the sum over the four lanes of quad mu
// (DPP quad permutations); K^2 likewise sums the quad's g_nu K_nu^2 partials (FP64).
// Spans and splits are compile-time loops, as in the direct form.
#pragma once

#include "bg_device.hpp"
#include "bg_group.hpp"
#include "bg_kernels.hpp"
#include "bg_split.hpp"

namespace bgk {

// sum over the four lanes of a quad, every lane receiving the total
template <typename T>
__device__ __forceinline__ T quad_sum(T x) {
#pragma clang fp contract(off)
  x = x + dpp_mov<kDppSwap1>(x);
  x = x + dpp_mov<kDppSwap2>(x);
  return x;
}

// LDS layout of one event's currents: [span][component][re, im] in T.
template <int L, typename T>
struct WCurrents {
  T* base;  // this event's block
  __device__ __forceinline__ T& re(int s, int c) const { return base[(s * 4 + c) * 2]; }
  __device__ __forceinline__ T& im(int s, int c) const { return base[(s * 4 + c) * 2 + 1]; }
  static constexpr int words = Spans<L>::count * 8;
};

// component c of a four-vector held in full, selected by bit masks (a chain of selects would
// be turned back into a dynamically indexed array on the stack)
template <typename U>
__device__ __forceinline__ U pick4(const U (&v)[4], int c) {
  using B = typename std::conditional<sizeof(U) == 8, uint64_t, uint32_t>::type;
  B r = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) r |= __builtin_bit_cast(B, v[k]) & (B)(-(B)(c == k));
  return __builtin_bit_cast(U, r);
}

// m = eps0 . V[0..L-1] by the W-tensor form, for the lanes (mu, nu) of one event group.
// kmu, knu: components mu, nu of the FP64 all-outgoing (scaled) momenta of the L recursion
// legs; emu, enu, e0mu: components of the sources and of the closing polarisation.
// Every lane of the group must call it with the same event (barriers inside).
template <int L, typename T>
__device__ __forceinline__ void bg_amplitude_w(int mu, int nu, const double (&kmu)[L], const double (&knu)[L],
                                               const T (&emu_re)[L], const T (&emu_im)[L], T e0mu_re, T e0mu_im,
                                               const WCurrents<L, T>& J, double& m_re, double& m_im) {
#pragma clang fp contract(off)
  using SP = Spans<L>;
  const T gnu = nu == 0 ? T(1) : T(-1);
  const T gmu = mu == 0 ? T(1) : T(-1);
  const double gnud = nu == 0 ? 1.0 : -1.0;
  // this lane's W_mu,nu and J_mu of every stored span
  T Wr[SP::count], Wi[SP::count], Jr[SP::count], Ji[SP::count];
  // single legs: J = eps, W = 2 eps_mu k_nu - k_mu eps_nu
  static_for<0, L>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    Jr[t] = emu_re[t];
    Ji[t] = emu_im[t];
    if (nu == 0) {
      J.re(t, mu) = emu_re[t];
      J.im(t, mu) = emu_im[t];
    }
  });
  __syncthreads();
  static_for<0, L>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    const T knut = T(knu[t]), kmut = T(kmu[t]);
    const T enr = J.re(t, nu), eni = J.im(t, nu);
    Wr[t] = fmac(T(2) * Jr[t], knut, -(kmut * enr));
    Wi[t] = fmac(T(2) * Ji[t], knut, -(kmut * eni));
  });
  T Vr = T(0), Vi = T(0);
  static_for<2, L + 1>([&](auto lc) {
    constexpr int len = decltype(lc)::value;
    static_for<0, L - len + 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value, b = a + len - 1, s = SP::at(a, b);
      // (W[B] . J[A] - W[A] . J[B])_mu: this lane's nu-term, then the quad sum
      T ar = T(0), ai = T(0);
      static_for<a, b>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int A = SP::at(a, i), B = SP::at(i + 1, b);
        const T jar = gnu * J.re(A, nu), jai = gnu * J.im(A, nu);
        const T jbr = gnu * J.re(B, nu), jbi = gnu * J.im(B, nu);
        ar = fmac(Wr[B], jar, ar);
        ar = fmac(-Wi[B], jai, ar);
        ai = fmac(Wr[B], jai, ai);
        ai = fmac(Wi[B], jar, ai);
        ar = fmac(-Wr[A], jbr, ar);
        ar = fmac(Wi[A], jbi, ar);
        ai = fmac(-Wr[A], jbi, ai);
        ai = fmac(-Wi[A], jbr, ai);
      });
      const T vr = quad_sum(ar), vi = quad_sum(ai);
      if constexpr (len < L) {
        // span momentum: components mu, nu (FP64 left-to-right sums), K^2 from the quad
        double Kmu = kmu[a], Knu = knu[a];
        static_for<a + 1, b + 1>([&](auto tc) {
          Kmu += kmu[decltype(tc)::value];
          Knu += knu[decltype(tc)::value];
        });
        const double k2 = quad_sum(gnud * (Knu * Knu));
        T prop;
        if constexpr (std::is_same<T, float>::value)
          prop = __builtin_amdgcn_rcpf(float(k2));
        else
          prop = 1.0 / k2;
        Jr[s] = vr * prop;
        Ji[s] = vi * prop;
        if (nu == 0) {
          J.re(s, mu) = Jr[s];
          J.im(s, mu) = Ji[s];
        }
        __syncthreads();
        // W[a..b] = 2 J_mu K_nu - K_mu J_nu + sum_i (J_mu[A] J_nu[B] - J_mu[B] J_nu[A])
        const T Knut = T(Knu), Kmut = T(Kmu);
        const T jnr = J.re(s, nu), jni = J.im(s, nu);
        T wr = fmac(T(2) * Jr[s], Knut, -(Kmut * jnr));
        T wi = fmac(T(2) * Ji[s], Knut, -(Kmut * jni));
        static_for<a, b>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int A = SP::at(a, i), B = SP::at(i + 1, b);
          const T bnr = J.re(B, nu), bni = J.im(B, nu), anr = J.re(A, nu), ani = J.im(A, nu);
          wr = fmac(Jr[A], bnr, wr);
          wr = fmac(-Ji[A], bni, wr);
          wi = fmac(Jr[A], bni, wi);
          wi = fmac(Ji[A], bnr, wi);
          wr = fmac(-Jr[B], anr, wr);
          wr = fmac(Ji[B], ani, wr);
          wi = fmac(-Jr[B], ani, wi);
          wi = fmac(-Ji[B], anr, wi);
        });
        Wr[s] = wr;
        Wi[s] = wi;
      } else {
        Vr = vr;
        Vi = vi;
      }
    });
  });
  // m = sum_mu g_mu eps0_mu V_mu: one lane per quad contributes, summed over the four quads
  T cr = T(0), ci = T(0);
  if (nu == 0) {
    cr = gmu * fmac(e0mu_re, Vr, -(e0mu_im * Vi));
    ci = gmu * fmac(e0mu_re, Vi, e0mu_im * Vr);
  }
  const int lane = (int)(threadIdx.x & 63u);
  cr = cr + __shfl(cr, lane ^ 4);
  ci = ci + __shfl(ci, lane ^ 4);
  cr = cr + __shfl(cr, lane ^ 8);
  ci = ci + __shfl(ci, lane ^ 8);
  m_re = double(cr);
  m_im = double(ci);
}

// |A(sigma;h)|^2 by the W-tensor form for the event of this lane's 16-lane group (position-
// ordered physical momenta, as ordered_amp2); J: the group's LDS block.
template <int N, typename T>
__device__ __forceinline__ double ordered_amp2_w(const double (&p)[N][4], const uint32_t (&leg)[N], uint32_t hel,
                                                 int mu, int nu, const WCurrents<N - 1, T>& J) {
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) esum += fabs(p[t][0]);
  const int ex = ilogb(0.5 * esum);
  const double sc = ldexp(1.0, -ex);
  double kmu[N - 1], knu[N - 1];
  T er[N - 1], ei[N - 1];
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = leg[t] < 2u ? -sc : sc;
    kmu[t - 1] = sg * pick4(p[t], mu);
    knu[t - 1] = sg * pick4(p[t], nu);
    const cv4<T> e = polarisation<T>(p[t], (hel >> leg[t]) & 1u);
    er[t - 1] = pick4(e.re, mu);
    ei[t - 1] = pick4(e.im, mu);
  }
  const cv4<T> e0 = polarisation<T>(p[0], (hel >> leg[0]) & 1u);
  double mr, mi;
  bg_amplitude_w<N - 1, T>(mu, nu, kmu, knu, er, ei, pick4(e0.re, mu), pick4(e0.im, mu), J, mr, mi);
  return ldexp(__builtin_fma(mr, mr, mi * mi), 2 * ex * (4 - N) - (N - 2));
}

// bg_amp2 with the W-tensor form.  Launch: 64-lane workgroups (four events of 16 lanes),
// ceil(count / 4) workgroups, 4 * WCurrents<N-1,T>::words * sizeof(T) bytes of dynamic LDS.
template <int N, typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_amp2_w(
    int64_t count, const double* __restrict__ mom, const uint32_t* __restrict__ hel, const uint8_t* __restrict__ order,
    double* __restrict__ out) {
  extern __shared__ unsigned char wlds[];
  const int grp = (int)(threadIdx.x >> 4), l = (int)(threadIdx.x & 15u);
  const int64_t i = (int64_t)blockIdx.x * 4 + grp;
  const int64_t ie = i < count ? i : count - 1;  // every group runs (barriers); only live ones store
  double p[N][4];
  uint32_t leg[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const uint32_t lg = order[ie * N + t];
    leg[t] = lg < (uint32_t)N ? lg : (uint32_t)(N - 1);  // malformed input stays in bounds
    const double* q = mom + (ie * N + leg[t]) * 4;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) p[t][mu] = q[mu];
  }
  const WCurrents<N - 1, T> J{reinterpret_cast<T*>(wlds) + grp * WCurrents<N - 1, T>::words};
  const double a2 = ordered_amp2_w<N, T>(p, leg, hel[ie], l >> 2, l & 3, J);
  if (l == 0 && i < count) out[i] = a2;
}

// The recursion kernel of the split generation with the W-tensor form: events first ..
// first + cnt - 1 from staging slots 0 .. cnt - 1 (k_kin<N>), 64 events per workgroup in
// 16 rounds of four; one compensated partial per 64 events, in event order.  Launch:
// 64-lane workgroups, ceil(cnt / 64) of them, first a multiple of 64, the dynamic LDS of
// k_amp2_w.
template <int N, typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rec_w(
    GenClass C, int64_t first, int64_t cnt, const double* __restrict__ buf, double* partials) {
  using L = SplitLayout<N>;
  extern __shared__ unsigned char wlds[];
  const int grp = (int)(threadIdx.x >> 4), l = (int)(threadIdx.x & 15u);
  const WCurrents<N - 1, T> J{reinterpret_cast<T*>(wlds) + grp * WCurrents<N - 1, T>::words};
  CSum w{0.0, 0.0}, w2{0.0, 0.0};
  for (int r = 0; r < 16; ++r) {
    const int64_t j = (int64_t)blockIdx.x * 64 + 4 * r + grp;
    const int64_t je = j < cnt ? j : cnt - 1;
    const double shat = buf[L::at(je, L::kShat)];
    double pc[N][4];
    const double hb = 0.5 * (C.use_pdf ? sqrt(shat) : C.sqrt_s);
    pc[0][0] = hb;
    pc[0][1] = 0.0;
    pc[0][2] = 0.0;
    pc[0][3] = hb;
#pragma unroll
    for (int t = 1; t < N; ++t)
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) pc[t][mu] = buf[L::at(je, L::kMom + 4 * (t - 1) + mu)];
    const uint64_t meta = (uint64_t)__double_as_longlong(buf[L::at(je, L::kMeta)]);
    const uint64_t legs = (uint64_t)__double_as_longlong(buf[L::at(je, L::kLegs)]);
    uint32_t leg[N];
#pragma unroll
    for (int t = 0; t < N; ++t) leg[t] = (uint32_t)(legs >> (4 * t)) & 15u;
    const double a2 = ordered_amp2_w<N, T>(pc, leg, (uint32_t)meta, l >> 2, l & 3, J);
    __syncthreads();  // the next round reuses the currents' LDS
    if (l == 0 && j < cnt) {
      const double x = finish_event<N>(C, first + j, ((meta >> 32) & 1u) != 0, a2, shat, buf[L::at(je, L::kX1)],
                                       buf[L::at(je, L::kX2)], buf[L::at(je, L::kR)]);
      w = cs_add(w, CSum{x, 0.0});
      w2 = cs_add(w2, CSum{x * x, 0.0});
    }
  }
  if (partials) block_reduce_store(w, w2, partials + 4 * (first / 64 + (int64_t)blockIdx.x));
}

template <int N, typename T>
constexpr unsigned w_lds_bytes() {
  return 4u * (unsigned)WCurrents<N - 1, T>::words * (unsigned)sizeof(T);
}

// k_kin<N> and k_rec_w<N, T> over the class in chunks of W.stage_cap events.
template <int N, typename T>
hipError_t launch_generate_w(const GenClass& C, const GenWork& W, hipStream_t s) {
  if (C.count <= 0) return hipSuccess;
  if (!W.stage || W.stage_cap < 64 || W.stage_cap % 64 != 0) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  for (int64_t first = 0; first < C.count && e == hipSuccess; first += W.stage_cap) {
    const int64_t cnt = std::min<int64_t>(W.stage_cap, C.count - first);
    hipLaunchKernelGGL((k_kin<N>), dim3((unsigned)((cnt + kKinBlock - 1) / kKinBlock)), dim3(kKinBlock),
                       perm_lds_bytes(N, kKinBlock), s, C, first, cnt, W.stage);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL((k_rec_w<N, T>), dim3((unsigned)((cnt + 63) / 64)), dim3(64), (w_lds_bytes<N, T>()), s, C,
                       first, cnt, W.stage, W.partials);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace bgk
