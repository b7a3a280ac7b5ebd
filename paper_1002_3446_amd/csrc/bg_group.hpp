// The recursion of Eqs. 3.1-3.2 and the closure of Eq. 3.6 with one event spread over G
// adjacent lanes of a wave (G = 2 or 4; the one-lane form is bg_amplitude).
//
// Lane g of a group holds the Lorentz components mu = g C .. g C + C - 1 (C = 4 / G) of
// every current and span scalar's share, so a lane needs about 1/G of the registers of
// the one-lane form; at n >= 10 in FP32 and n >= 7 in FP64 the one-lane form exceeds the
// 512 registers a lane can address and spills to scratch memory.  Minkowski products are
// formed per lane over its components with their metric signs sigma_mu = (+,-,-,-) and
// completed across the group by DPP lane permutations; every lane of the group ends with
// the bitwise same total (IEEE addition is commutative), so the group stays consistent.
//
// Span momenta enter covariantly, K_mu = sigma_mu K^mu: the FP64 leg momenta are signed
// once per event, so J.K needs no signs, and the K-dependent part of a bracket is summed
// covariantly and converted to contravariant once per span.  K^2 is the group sum of the
// lanes' FP64 partials sigma_mu K_mu^2.
#pragma once

#include "bg_device.hpp"

namespace bgk {

template <typename T, int C>
struct cvl {
  T re[C], im[C];
};

// DPP quad permutations: swap neighbouring lanes, swap neighbouring lane pairs
constexpr int kDppSwap1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppSwap2 = 0x4E;  // quad_perm [2, 3, 0, 1]

// (old value 0 with bound_ctrl: the FP32 form folds into v_add_f32_dpp)
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the G lanes of a group; every lane receives the same total.  (Kept apart from
// neighbouring products so that the FP32 add takes its operand through DPP.)
template <int G, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma clang fp contract(off)
  if constexpr (G >= 2) x = x + dpp_mov<kDppSwap1>(x);
  if constexpr (G >= 4) x = x + dpp_mov<kDppSwap2>(x);
  return x;
}

// This lane's share of a group: its first component and the metric signs of its components.
template <int G, typename T>
struct LaneShare {
  static constexpr int C = 4 / G;
  int mu0;     // first component held
  T sg[C];     // sigma of each held component
  __device__ __forceinline__ explicit LaneShare(int g) : mu0(g * C) {
#pragma unroll
    for (int c = 0; c < C; ++c) sg[c] = (mu0 + c == 0) ? T(1) : T(-1);
  }
  // the held components of a full four-vector, without dynamic register indexing: one select
  // for two lanes in the forward kernels; bit masks for four lanes, and for two in the
  // gradient kernels (BITS), where selects between elements of one array are turned back into
  // a dynamically indexed array on the stack
  template <bool BITS = false, typename U>
  __device__ __forceinline__ U pick(const U (&v)[4], int c) const {
    if constexpr (G == 4 || BITS) {
      using B = typename std::conditional<sizeof(U) == 8, uint64_t, uint32_t>::type;
      B r = 0;
#pragma unroll
      for (int q = 0; q < G; ++q) r |= __builtin_bit_cast(B, v[q * C + c]) & (B)(-(B)(mu0 == q * C));
      return __builtin_bit_cast(U, r);
    } else {
      U r = v[c];
#pragma unroll
      for (int q = 1; q < G; ++q) r = (mu0 == q * C) ? v[q * C + c] : r;
      return r;
    }
  }
};

// DPP control that gives every lane of a group of G adjacent lanes the value of the group's
// lane K (a quad permutation: [K, K, K, K] for G = 4, [K, K, 2 + K, 2 + K] for G = 2).
template <int G, int K>
constexpr int group_bcast_ctrl() {
  return G == 4 ? (K | (K << 2) | (K << 4) | (K << 6)) : (K | (K << 2) | ((2 + K) << 4) | ((2 + K) << 6));
}

template <int G, int K, typename T>
__device__ __forceinline__ T group_bcast(T x) {
  if constexpr (G == 1) {
    return x;
  } else if constexpr (std::is_same<T, float>::value) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), group_bcast_ctrl<G, K>(),
                                                              0xF, 0xF, false));
  } else {
    return dpp_mov<group_bcast_ctrl<G, K>()>(x);
  }
}

// Whether a group keeps its span scalars distributed over its lanes: where the currents of
// every span already take most of a lane's registers (FP32 n = 12 with two lanes, FP64 from
// n = 9), replicating the scalars on every lane would spill.
template <int L, int G, typename T>
constexpr bool dist_scalars() {
  return G > 1 && Spans<L>::count * 2 * (4 / G) * (int)(sizeof(T) / 4) > 240;
}

// The span scalars S of a group (the complex sums of the three-gluon dots, one per span of
// two or more legs; spans counted from the first of two legs, q = s - L).  Replicated: every
// lane holds every scalar.  Distributed: lane q % G of the group holds span q in slot q / G,
// and a read broadcasts it over the group (one DPP move per word); writes of a group-uniform
// value go to the owning lane by a select.  Either way every lane reads bitwise the value
// that was written.
template <int L, int G, typename T, bool DIST = dist_scalars<L, G, T>()>
struct SpanScalars {
  static constexpr int kCount = Spans<L>::count - L;
  static constexpr int kSlots = DIST ? (kCount + G - 1) / G : kCount;
  T re[kSlots], im[kSlots];
  int g;  // this lane's place in its group
  __device__ __forceinline__ explicit SpanScalars(int g_) : g(g_) {}
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int m = 0; m < kSlots; ++m) re[m] = im[m] = T(0);
  }
  template <int S>
  __device__ __forceinline__ void get(T& r, T& i) const {
    constexpr int q = S - L;
    static_assert(q >= 0 && q < kCount, "span scalar index");
    if constexpr (DIST) {
      r = group_bcast<G, q % G>(re[q / G]);
      i = group_bcast<G, q % G>(im[q / G]);
    } else {
      r = re[q];
      i = im[q];
    }
  }
  template <int S>
  __device__ __forceinline__ void put(T r, T i) {
    constexpr int q = S - L;
    static_assert(q >= 0 && q < kCount, "span scalar index");
    if constexpr (DIST) {
      const bool own = g == q % G;
      re[q / G] = own ? r : re[q / G];
      im[q / G] = own ? i : im[q / G];
    } else {
      re[q] = r;
      im[q] = i;
    }
  }
  // S -= (r, i) for a group-uniform (r, i)
  template <int S>
  __device__ __forceinline__ void sub(T r, T i) {
    constexpr int q = S - L;
    static_assert(q >= 0 && q < kCount, "span scalar index");
    if constexpr (DIST) {
      const bool own = g == q % G;
      re[q / G] = own ? re[q / G] - r : re[q / G];
      im[q / G] = own ? im[q / G] - i : im[q / G];
    } else {
      re[q] -= r;
      im[q] -= i;
    }
  }
};

// x.y over the group (bilinear, metric (+,-,-,-))
template <int G, typename T, int C>
__device__ __forceinline__ void cdot_g(const LaneShare<G, T>& ls, const cvl<T, C>& x, const cvl<T, C>& y, T& r,
                                       T& i) {
  r = ls.sg[0] * fmac(-x.im[0], y.im[0], x.re[0] * y.re[0]);
  i = ls.sg[0] * fmac(x.im[0], y.re[0], x.re[0] * y.im[0]);
#pragma unroll
  for (int c = 1; c < C; ++c) {
    r = fmac(ls.sg[c], fmac(-x.im[c], y.im[c], x.re[c] * y.re[c]), r);
    i = fmac(ls.sg[c], fmac(x.im[c], y.re[c], x.re[c] * y.im[c]), i);
  }
  r = group_sum<G>(r);
  i = group_sum<G>(i);
}

// x.K over the group for a covariant real K (this lane's components)
template <int G, typename T, int C>
__device__ __forceinline__ void rdot_g(const cvl<T, C>& x, const T (&k)[C], T& r, T& i) {
  r = x.re[0] * k[0];
  i = x.im[0] * k[0];
#pragma unroll
  for (int c = 1; c < C; ++c) {
    r = fmac(x.re[c], k[c], r);
    i = fmac(x.im[c], k[c], i);
  }
  r = group_sum<G>(r);
  i = group_sum<G>(i);
}

template <typename T, int C>
__device__ __forceinline__ void caxpy_l(T cr, T ci, const cvl<T, C>& y, cvl<T, C>& acc) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    acc.re[c] = fmac(-ci, y.im[c], fmac(cr, y.re[c], acc.re[c]));
    acc.im[c] = fmac(ci, y.re[c], fmac(cr, y.im[c], acc.im[c]));
  }
}

// Covariant span momenta of this lane's components, summed left to right in FP64 over the
// legs and cast to T; propagators 1/K^2 from the group sum of FP64 partials.
template <int L, int G, typename T, bool AFRESH = false>
struct SpanKGroup {
  static constexpr int C = 4 / G;
  const double (&k)[L][C];   // covariant FP64 leg components held by this lane
  const double (&sg)[C];     // their metric signs
  // With AFRESH, every use sums afresh: an optimisation barrier on the first term keeps the
  // compiler from merging the sums of one span over the whole kernel and holding them in
  // registers (the gradient kernels, which hold currents and adjoints, and the FP64 forward
  // forms that would otherwise spill gain registers; elsewhere the forward kernels lose more
  // to the extra FP64 adds than they gain).
  template <int A, int B>
  __device__ __forceinline__ void sum(double d[C]) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      d[c] = k[A][c];
      if constexpr (AFRESH) opaque(d[c]);
    }
    static_for<A + 1, B + 1>([&](auto t) {
#pragma unroll
      for (int c = 0; c < C; ++c) d[c] += k[decltype(t)::value][c];
    });
  }
  template <int A, int B>
  __device__ __forceinline__ void K(T (&out)[C]) const {
    double d[C];
    sum<A, B>(d);
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = T(d[c]);
  }
  template <int A, int B>
  __device__ __forceinline__ T prop() const {
    double d[C];
    sum<A, B>(d);
    double part;
    {
#pragma clang fp contract(off)
      part = sg[0] * (d[0] * d[0]);
#pragma unroll
      for (int c = 1; c < C; ++c) part = part + sg[c] * (d[c] * d[c]);
    }
    const double k2 = group_sum<G>(part);
    if constexpr (std::is_same<T, float>::value)
      return __builtin_amdgcn_rcpf(float(k2));
    else
      return 1.0 / k2;
  }
};

// The same span momenta read from a per-workgroup LDS table filled once per event: for every
// span of 2..L-1 legs this lane's covariant components, summed left to right in FP64 over
// its legs and cast to T (bitwise the values SpanKGroup forms at each use), layout
// [span][component][lane] so that a wave's reads are contiguous.  Single legs and the
// propagators still come from the FP64 leg momenta.  One table read replaces the FP64 sums
// and conversions at every use, and nothing of the sums stays live in registers.
template <int L, int G, typename T>
struct SpanKGroupLds : SpanKGroup<L, G, T> {
  using Base = SpanKGroup<L, G, T>;
  static constexpr int C = Base::C;
  static constexpr int kSpans = Spans<L>::count - L - 1;  // spans of 2..L-1 legs
  T* kt;      // &table[0][0][lane]
  int lanes;  // lanes per workgroup (the table's row stride)
  __device__ __forceinline__ SpanKGroupLds(const double (&k_)[L][C], const double (&sg_)[C], T* kt_, int lanes_)
      : Base{k_, sg_}, kt(kt_), lanes(lanes_) {}
  __device__ __forceinline__ void fill() const {
    using SP = Spans<L>;
    static_for<0, L - 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      double acc[C];
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = this->k[a][c];
      static_for<a + 1, L>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += this->k[b][c];
        if constexpr (b - a + 1 < L) {
          constexpr int q = SP::at(a, b) - L;
#pragma unroll
          for (int c = 0; c < C; ++c) kt[(q * C + c) * lanes] = T(acc[c]);
        }
      });
    });
    // the recursion reads the table back instead of keeping the values in registers
    asm volatile("" ::: "memory");
  }
  template <int A, int B>
  __device__ __forceinline__ void K(T (&out)[C]) const {
    if constexpr (A == B) {
#pragma unroll
      for (int c = 0; c < C; ++c) out[c] = T(this->k[A][c]);
    } else {
      constexpr int q = Spans<L>::at(A, B) - L;
      static_assert(q >= 0 && q < kSpans, "span of 2..L-1 legs");
#pragma unroll
      for (int c = 0; c < C; ++c) out[c] = kt[(q * C + c) * lanes];
    }
  }
};

// LDS bytes per lane of SpanKGroupLds
template <int L, int G, typename T>
constexpr int span_k_lds_bytes() {
  return SpanKGroupLds<L, G, T>::kSpans * (4 / G) * (int)sizeof(T);
}

// One span [A..B]: its bracket sum V (contravariant, this lane's components).
template <int L, int A, int B, int G, typename T, typename KS, typename SS>
__device__ __forceinline__ void span_vertex_g(const LaneShare<G, T>& ls, const KS& ks,
                                              const cvl<T, 4 / G> (&J)[Spans<L>::count], const SS& S,
                                              cvl<T, 4 / G>& V, T& sr, T& si) {
  constexpr int C = 4 / G;
  using SP = Spans<L>;
  cvl<T, C> X, Z, Yc;  // (J.K) J terms, S terms (contravariant); d (K_A - K_B) (covariant)
#pragma unroll
  for (int c = 0; c < C; ++c) X.re[c] = X.im[c] = Z.re[c] = Z.im[c] = Yc.re[c] = Yc.im[c] = T(0);
  sr = T(0);
  si = T(0);
  static_for<A, B>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int PA = SP::at(A, i), PB = SP::at(i + 1, B);
    T ka[C], kb[C];
    ks.template K<A, i>(ka);
    ks.template K<i + 1, B>(kb);
    T dr, di, ar, ai, br, bi;
    cdot_g<G>(ls, J[PA], J[PB], dr, di);
    rdot_g<G>(J[PA], kb, ar, ai);
    rdot_g<G>(J[PB], ka, br, bi);
    caxpy_l(ar, ai, J[PB], X);
    caxpy_l(-br, -bi, J[PA], X);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const T dk = ka[c] - kb[c];
      Yc.re[c] = fmac(dr, dk, Yc.re[c]);
      Yc.im[c] = fmac(di, dk, Yc.im[c]);
    }
    sr += dr;
    si += di;
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<i + 1, B>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      T dr, di;
      cdot_g<G>(ls, J[SP::at(A, i)], J[SP::at(j + 1, B)], dr, di);
      caxpy_l(dr, di, J[SP::at(i + 1, j)], X);
    });
  });
  static_for<A + 1, B>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    T r, i;
    S.template get<SP::at(A, j)>(r, i);
    caxpy_l(-r, -i, J[SP::at(j + 1, B)], Z);
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    T r, im;
    S.template get<SP::at(i + 1, B)>(r, im);
    caxpy_l(-r, -im, J[SP::at(A, i)], Z);
  });
#pragma unroll
  for (int c = 0; c < C; ++c) {
    V.re[c] = fmac(T(2), X.re[c], fmac(ls.sg[c], Yc.re[c], Z.re[c]));
    V.im[c] = fmac(T(2), X.im[c], fmac(ls.sg[c], Yc.im[c], Z.im[c]));
  }
}

// Forward recursion: every stored current and span scalar, and the undivided bracket sum V
// of the full span (this lane's components).
template <int L, int G, typename T, typename KS, typename SS>
__device__ __forceinline__ void bg_forward_g(const LaneShare<G, T>& ls, const KS& ks,
                                             const cvl<T, 4 / G> (&src)[L], cvl<T, 4 / G> (&J)[Spans<L>::count],
                                             SS& S, cvl<T, 4 / G>& Vfull) {
  constexpr int C = 4 / G;
  using SP = Spans<L>;
  static_for<0, L>([&](auto ac) { J[decltype(ac)::value] = src[decltype(ac)::value]; });
  static_for<2, L>([&](auto lc) {
    constexpr int len = decltype(lc)::value;
    static_for<0, L - len + 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value, b = a + len - 1, s = SP::at(a, b);
      cvl<T, C> V;
      T sr, si;
      span_vertex_g<L, a, b, G, T>(ls, ks, J, S, V, sr, si);
      const T prop = ks.template prop<a, b>();
#pragma unroll
      for (int c = 0; c < C; ++c) {
        J[s].re[c] = V.re[c] * prop;
        J[s].im[c] = V.im[c] * prop;
      }
      S.template put<s>(sr, si);
    });
  });
  T sr, si;
  span_vertex_g<L, 0, L - 1, G, T>(ls, ks, J, S, Vfull, sr, si);
}

// Forward recursion and closure m = eps0 . V[0..L-1] (every lane of the group gets m).
template <int L, int G, typename T, typename KS>
__device__ __forceinline__ void bg_amplitude_g(const LaneShare<G, T>& ls, const KS& ks,
                                               const cvl<T, 4 / G> (&src)[L], const cvl<T, 4 / G>& eps0,
                                               double& m_re, double& m_im) {
  constexpr int C = 4 / G;
  using SP = Spans<L>;
  cvl<T, C> J[SP::count];
  SpanScalars<L, G, T> S(ls.mu0 / C);
  cvl<T, C> V;
  bg_forward_g<L, G, T>(ls, ks, src, J, S, V);
  T mr, mi;
  cdot_g<G>(ls, eps0, V, mr, mi);
  m_re = double(mr);
  m_im = double(mi);
}

}  // namespace bgk
