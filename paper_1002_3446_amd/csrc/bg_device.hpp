// Device building blocks of the event path, one event per lane (gfx950).
//
// Paper: Giele, Stavenga, Winter, "Thread-Scalable Evaluation of Multi-Jet Observables".
//   philox4x32        counter-based draws (generator unnamed in the paper, Sec. 4)
//   pdf_sample2       synthetic gluon density x^a (1-x)^b by inverse CDF (stands in for
//                     the LHAPDF grids of Sec. 3)
//   rambo_q/rambo_map RAMBO massless phase space (Sec. 3)
//   polarisation      helicity sources J[i] orthogonal to k_i (Sec. 3)
//   bg_amplitude      Berends-Giele recursion (Eqs. 3.1, 3.2) and amputated closure (Eq. 3.6)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "bg_math.hpp"

namespace bgk {

// Compile-time loop: f(integral_constant<int, I>) for I = B .. E-1.  Every index of the
// recursion is a constant after instantiation, so the per-lane arrays are scalarised into
// registers independently of the compiler's unrolling heuristics.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ----------------------------------------------------------------------------------------
// Philox-4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies, key
// advanced by the Weyl constants between rounds.
// ----------------------------------------------------------------------------------------
struct u32x4 {
  uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32x32 -> 64-bit product as one v_mad_u64_u32 rather than separate low and high
    // multiplies (both forms are quarter-rate instructions)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return u32x4{{c0, c1, c2, c3}};
}

// word -> (r + 1/2) 2^-32, exact in double and strictly inside (0, 1)
__device__ __forceinline__ double u01(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }

// Draw layout of one event: counter (block, event lo, event hi, n), key (seed lo, seed hi).
//   block 0: x1 uniform, x2 uniform, helicity word, unused
//   block 1 + p: rho1..rho4 of outgoing gluon p (leg p + 2)
//   block n - 1 + k/4, word k%4: shuffle word consumed at Fisher-Yates step t = n-2-k
struct EventRng {
  uint32_t e0, e1, n, k0, k1;
  __device__ __forceinline__ u32x4 block(uint32_t b) const { return philox4x32(b, e0, e1, n, k0, k1); }
};

// ----------------------------------------------------------------------------------------
// Colour ordering as nibbles: nibble i holds the leg at recursion position i+1 (legs 1..n-1).
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t nib(uint64_t A, int i) { return (uint32_t)(A >> (4 * i)) & 15u; }
__device__ __forceinline__ uint64_t set_nib(uint64_t A, int i, uint32_t v) {
  const uint64_t m = 15ull << (4 * i);
  return (A & ~m) | ((uint64_t)v << (4 * i));
}

template <int N>
__device__ __forceinline__ uint64_t identity_order() {
  uint64_t A = 0;
#pragma unroll
  for (int i = 0; i < N - 1; ++i) A |= (uint64_t)(i + 1) << (4 * i);
  return A;
}

// Fisher-Yates over positions 0..N-2 of the nibble list: for t = N-2 .. 1,
// j = (r_t (t+1)) >> 32, swap entries t and j (Sec. 3: random permutation of legs 2..n).
template <int N>
__device__ __forceinline__ uint64_t shuffle_order(const EventRng& rng) {
  uint64_t A = identity_order<N>();
  constexpr int NF = N - 2;
  u32x4 w{};
#pragma unroll
  for (int k = 0; k < N - 2; ++k) {
    if ((k & 3) == 0) w = rng.block(1 + NF + k / 4);
    const int t = N - 2 - k;
    const uint32_t r = w.v[k & 3];
    const uint32_t j = (uint32_t)(((uint64_t)r * (uint64_t)(t + 1)) >> 32);
    const uint32_t vt = nib(A, t), vj = nib(A, (int)j);
    A = set_nib(A, t, vj);
    A = set_nib(A, (int)j, vt);
  }
  return A;
}

// ----------------------------------------------------------------------------------------
// Synthetic density f(x) = x^a (1-x)^b, b integer, with primitive F(x) = x^(a+1) P(x),
// P(x) = sum_k C(b,k) (-1)^k x^k / (a+k+1), on [tau, 1); Z = F(1) - F(tau).  x = F^-1(u):
//
// Per event: a cubic from a per-class table gives x to ~1e-4 relative; then Newton steps
// on F(x) - F(tau) = u Z (u <= 1/2) or F(1) - F(x) = (1 - u) Z (u > 1/2), at least two and
// until the step is below 1e-7 relative (from the table's accuracy: two).  One log and
// one exp give w = x^(a+1) at the table point; each step moves x by x d and w by the
// binomial series of (1 + d)^(a+1) to fourth order, exact in FP64 for |d| < 1e-3
// (a larger step recomputes w).
//
// The table: u in [0, 1/2] in kPdfLowSeg equal segments; u > 1/2 by the binade of
// s = 1 - u in [2^-33, 1/2) (kPdfBinades of them, each in kPdfSub equal parts of its
// mantissa), which resolves the (1 - u)^(1/(b+1)) behaviour of x near 1.  Each segment
// holds the cubic Hermite interpolant of x in the local coordinate theta in [0, 1), from
// x and dx/dtheta = (Z / f(x)) du/dtheta at its ends; the ends are solved by pdf_solve.
// The host builds the table once per (a, b, tau) and device.
// ----------------------------------------------------------------------------------------
constexpr int kPdfLowSeg = 64;
constexpr int kPdfBinades = 32;  // s in [2^-33, 2^-1)
constexpr int kPdfSub = 8;
constexpr int kPdfSegs = kPdfLowSeg + kPdfBinades * kPdfSub;

struct PdfParams {
  double a, tau, Ftau, F1, Z, x0base;  // x0base = tau^(a+1)
  double usplit, xsplit;
  double coef[17];
  int b;
  const double* tab;  // [kPdfSegs][4] cubic coefficients (device memory)
};

__host__ __device__ inline double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

__host__ __device__ inline double pdf_poly(const PdfParams& P, double x) {
  double poly = P.coef[P.b];
  for (int k = P.b - 1; k >= 0; --k) poly = fma(poly, x, P.coef[k]);
  return poly;
}

// Robust solve of one table node (table setup only).  Newton's method in variables where the
// equation is nearly linear:
//   x < x_split (u < u_split):  log(F(x) - F(tau)) = log(u Z)        in y = log x,
//                               then one plain Newton step in x (x close to tau);
//   x >= x_split:               log(F(1) - F(x))   = log((1 - u) Z)  in z = log(1 - x);
// s = 1 - u is passed exactly.  Converges in 3..7 steps; at most 40.
__host__ __device__ inline double pdf_solve(double u, double s, const PdfParams& P) {
  if (u <= 0.0) return P.tau;
  const double ap1 = P.a + 1.0;
  const bool lower = u < P.usplit;
  double v, target;
  if (lower) {
    const double T = u * P.Z;
    target = log(T);
    const double base = P.x0base + ap1 * T;  // leading power only
    const double lx = base > 0.0 ? log(base) / ap1 : log(P.xsplit);
    v = fmin(fmax(lx, log(P.tau) + 1e-12), log(P.xsplit));
  } else {
    target = log(s * P.Z);
    v = -0.69314718055994530942;  // x = 1/2
  }
  for (int it = 0; it < 40; ++it) {
    const double e = exp(v);
    const double x = lower ? e : 1.0 - e;
    const double lx = lower ? v : log1p(-e);
    const double xa1 = exp(ap1 * lx);
    const double F = xa1 * pdf_poly(P, x);
    const double G = lower ? F - P.Ftau : P.F1 - F;
    const double omx_b = ipow(1.0 - x, P.b);
    // d log G / dv = x f / G (lower) or (1 - x) f / G (upper), with f = x^a (1-x)^b
    const double dG = lower ? xa1 * omx_b : xa1 / x * omx_b * (1.0 - x);
    if (!(G > 0.0)) {  // stepped outside the domain: restart inside it
      v = lower ? log(P.tau) + 1e-9 : -0.69314718055994530942;
      continue;
    }
    const double step = (log(G) - target) * G / dG;
    v -= step;
    if (fabs(step) <= 1e-9) break;
  }
  double x = lower ? exp(v) : 1.0 - exp(v);
  if (lower) {  // one plain Newton step in x: exact where x is close to tau
    const double xa1 = exp(ap1 * v);
    const double f = xa1 / x * ipow(1.0 - x, P.b);
    x -= (xa1 * pdf_poly(P, x) - P.Ftau - u * P.Z) / f;
  }
  return x;
}

// Segment and local coordinate of u (see above).  u <= 1/2 uses u itself; u > 1/2 the exact
// s = 1 - u, split by frexp into binade and mantissa.
__device__ __forceinline__ int pdf_segment(double u, double& theta) {
  if (u <= 0.5) {
    const double t = u * (2 * kPdfLowSeg);
    const int k = min(max((int)t, 0), kPdfLowSeg - 1);
    theta = t - k;
    return k;
  }
  int e;
  const double m = frexp(1.0 - u, &e);  // 1 - u = m 2^e, m in [1/2, 1)
  const int bin = min(max(e + 32, 0), kPdfBinades - 1);  // e = -32 .. -1 for s in [2^-33, 1/2)
  const double t = (ldexp(1.0 - u, 33 - bin) - 1.0) * kPdfSub;  // s / 2^(bin-33) in [1, 2)
  const int j = min(max((int)t, 0), kPdfSub - 1);
  theta = t - j;
  return kPdfLowSeg + bin * kPdfSub + j;
}

// u of a segment's local coordinate (the inverse of pdf_segment), with s = 1 - u exact
__host__ __device__ inline void pdf_node(int seg, double theta, double& u, double& s, double& dudtheta) {
  if (seg < kPdfLowSeg) {
    u = (seg + theta) / (2 * kPdfLowSeg);
    s = 1.0 - u;
    dudtheta = 1.0 / (2 * kPdfLowSeg);
    return;
  }
  const int bin = (seg - kPdfLowSeg) / kPdfSub, j = (seg - kPdfLowSeg) % kPdfSub;
  const double scale = ldexp(1.0, bin - 33);  // binade [2^(bin-33), 2^(bin-32))
  s = (1.0 + (j + theta) / kPdfSub) * scale;
  u = 1.0 - s;
  dudtheta = -scale / kPdfSub;
}

// x = F^-1(u) for one parton (see above).
__device__ __forceinline__ double pdf_sample(double u, const PdfParams& P) {
  const double A = P.a + 1.0;
  double theta;
  const int seg = pdf_segment(u, theta);
  const double* c = P.tab + 4 * seg;
  double x = fma(fma(fma(c[3], theta, c[2]), theta, c[1]), theta, c[0]);
  x = fmin(fmax(x, P.tau), 1.0 - 0x1p-53);
  double w = exp(A * log_fp64(x));
  const bool lower = u <= 0.5;
  const double uZ = lower ? u * P.Z : (1.0 - u) * P.Z;
  const double c1 = A, c2 = A * (A - 1.0) / 2.0, c3 = c2 * (A - 2.0) / 3.0, c4 = c3 * (A - 3.0) / 4.0;
  double d = 1.0;
  for (int it = 0; it < 8 && (it < 2 || fabs(d) > 1e-7); ++it) {
    const double F = w * pdf_poly(P, x);
    const double res = lower ? (F - P.Ftau) - uZ : uZ - (P.F1 - F);
    // Newton: dx = -res / f(x), f = (w / x) (1 - x)^b, so d = dx / x = -res / (w (1 - x)^b)
    d = -res / (w * ipow(1.0 - x, P.b));
    x = fma(x, d, x);
    if (fabs(d) < 1e-3) {
      w *= 1.0 + d * (c1 + d * (c2 + d * (c3 + d * c4)));
    } else {
      x = fmin(fmax(x, P.tau), 1.0 - 0x1p-53);
      w = exp(A * log_fp64(x));
    }
  }
  return x;
}

// One segment of the table (host side, once per density and device).
__host__ __device__ inline void pdf_table_segment(const PdfParams& P, int seg, double* out) {
  double u0, s0, du0, u1, s1, du1;
  pdf_node(seg, 0.0, u0, s0, du0);
  pdf_node(seg, 1.0, u1, s1, du1);
  const double x0 = pdf_solve(u0, s0, P), x1 = pdf_solve(u1, s1, P);
  const double f0 = exp(P.a * log(x0)) * ipow(1.0 - x0, P.b), f1 = exp(P.a * log(x1)) * ipow(1.0 - x1, P.b);
  const double d0 = P.Z / f0 * du0, d1 = P.Z / f1 * du1;  // dx/dtheta at the ends
  out[0] = x0;
  out[1] = d0;
  out[2] = 3.0 * (x1 - x0) - 2.0 * d0 - d1;
  out[3] = 2.0 * (x0 - x1) + d0 + d1;
}

// ----------------------------------------------------------------------------------------
// Running coupling and scale-dependent density on grids (Sec. 3: alpha_s on a 1-D grid in the
// renormalisation scale, the densities on a 2-D grid in factorisation scale and x, read with
// linear interpolation).  With a dynamic scale mu (= H_T of the event, Sec. 4) the weight
// takes alpha_s(mu)^(n-2) f(x1, mu) f(x2, mu) instead of alpha_s^(n-2) f(x1) f(x2).  The
// grids hold alpha_s at nodes uniform in ln mu and ln f at nodes uniform in (ln mu, y) with
// y = ln(x / (1 - x)), in which ln f is smooth at both ends of x; a point between nodes
// takes the linear (1-D) or bilinear (2-D) interpolation of the node values, evaluated in
// FP64 as written; scales and x outside the grids take the edge values.
// ----------------------------------------------------------------------------------------
constexpr int kAlphaNodes = 512;
constexpr int kGridMuNodes = 64;
constexpr int kGridYNodes = 1024;
constexpr double kGridMuLo = 5.0, kGridMuHi = 20000.0;  // GeV
constexpr double kGridXLo = 1e-6, kGridXHi = 1.0 - 1e-9;

struct ScaleGrid {
  const double* alpha;  // [kAlphaNodes]
  const double* lnf;    // [kGridMuNodes][kGridYNodes]
  double lmu_lo, dlmu_alpha, dlmu_pdf, y_lo, dy;
};

// node index and fraction of v on a uniform grid of n nodes from lo with spacing h
__host__ __device__ inline int grid_cell(double v, double lo, double h, int n, double& t) {
#pragma clang fp contract(off)
  double s = (v - lo) / h;
  s = s < 0.0 ? 0.0 : (s > (double)(n - 1) ? (double)(n - 1) : s);
  int i = (int)s;
  i = i > n - 2 ? n - 2 : i;
  t = s - (double)i;
  return i;
}

__host__ __device__ inline double grid_alpha(const ScaleGrid& g, double lmu) {
#pragma clang fp contract(off)
  double t;
  const int i = grid_cell(lmu, g.lmu_lo, g.dlmu_alpha, kAlphaNodes, t);
  return (1.0 - t) * g.alpha[i] + t * g.alpha[i + 1];
}

__host__ __device__ inline double grid_lnf(const ScaleGrid& g, double lmu, double y) {
#pragma clang fp contract(off)
  double tm, ty;
  const int im = grid_cell(lmu, g.lmu_lo, g.dlmu_pdf, kGridMuNodes, tm);
  const int iy = grid_cell(y, g.y_lo, g.dy, kGridYNodes, ty);
  const double* r0 = g.lnf + (size_t)im * kGridYNodes + iy;
  const double* r1 = r0 + kGridYNodes;
  const double f0 = (1.0 - ty) * r0[0] + ty * r0[1];
  const double f1 = (1.0 - ty) * r1[0] + ty * r1[1];
  return (1.0 - tm) * f0 + tm * f1;
}

// ----------------------------------------------------------------------------------------
// RAMBO (Sec. 3).  From (rho1..rho4): c = 2 rho1 - 1, phi = 2 pi rho2, q0 = -ln(rho3 rho4),
// q = q0 (sin cos phi, sin sin phi, c).  Then the conformal map with Q = sum q.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ void rambo_q(double r1, double r2, double r3, double r4, double q[4]) {
  const double c = 2.0 * r1 - 1.0;
  const double st = sqrt(1.0 - c * c);
  double sp, cp;
  sincospi_fp64(2.0 * r2, &sp, &cp);
  const double q0 = -log_fp64(r3 * r4);
  q[0] = q0;
  q[1] = q0 * st * cp;
  q[2] = q0 * st * sp;
  q[3] = q0 * c;
}

struct RamboMap {
  double bx, by, bz, gamma, a, X;
  __device__ __forceinline__ void init(const double Q[4], double sqrt_shat) {
    const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    const double iM = 1.0 / M;
    bx = -Q[1] * iM;
    by = -Q[2] * iM;
    bz = -Q[3] * iM;
    gamma = Q[0] * iM;
    a = 1.0 / (1.0 + gamma);
    X = sqrt_shat * iM;
  }
  __device__ __forceinline__ void apply(const double q[4], double p[4]) const {
    const double bq = bx * q[1] + by * q[2] + bz * q[3];
    p[0] = X * (gamma * q[0] + bq);
    p[1] = X * (q[1] + bx * q[0] + a * bq * bx);
    p[2] = X * (q[2] + by * q[0] + a * bq * by);
    p[3] = X * (q[3] + bz * q[0] + a * bq * bz);
  }
};

// ----------------------------------------------------------------------------------------
// Complex four-vectors and the helicity sources.
// ----------------------------------------------------------------------------------------
template <typename T>
struct cv4 {
  T re[4], im[4];
};

// eps_h(p) = (0, -h ct cf + i sf, -h ct sf - i cf, h st) / sqrt(2) from the physical momentum,
// evaluated in the recursion precision T (the vector only enters the recursion in T).
// In FP32 the two inverse lengths come from the hardware reciprocal square root (about
// one ulp), in FP64 from correctly rounded square roots and divisions.
template <typename T>
__device__ __forceinline__ cv4<T> polarisation(const double p[4], bool plus) {
  // no implicit fused multiply-adds: the vector rounds as written in every kernel
#pragma clang fp contract(off)
  const T px = T(p[1]), py = T(p[2]), pz = T(p[3]);
  const T pt2 = px * px + py * py;
  T ct, st, cf = T(1), sf = T(0);
  if constexpr (std::is_same<T, float>::value) {
    const float ipa = __builtin_amdgcn_rsqf(pt2 + pz * pz);
    const float ipt = __builtin_amdgcn_rsqf(pt2);
    ct = pz * ipa;
    st = pt2 > 0.0f ? (pt2 * ipt) * ipa : 0.0f;
    if (pt2 > 0.0f) {
      cf = px * ipt;
      sf = py * ipt;
    }
  } else {
    const T pa = sqrt(pt2 + pz * pz);
    const T pt = sqrt(pt2);
    const T ipa = T(1) / pa;
    ct = pz * ipa;
    st = pt * ipa;
    if (pt2 > T(0)) {
      const T ipt = T(1) / pt;
      cf = px * ipt;
      sf = py * ipt;
    }
  }
  const T r = T(0.70710678118654752440);
  const T h = plus ? r : -r;
  cv4<T> e;
  e.re[0] = T(0);
  e.im[0] = T(0);
  e.re[1] = -h * ct * cf;
  e.im[1] = sf * r;
  e.re[2] = -h * ct * sf;
  e.im[2] = -cf * r;
  e.re[3] = h * st;
  e.im[3] = T(0);
  return e;
}

// ----------------------------------------------------------------------------------------
// Berends-Giele recursion, Eqs. 3.1-3.2, over L ordered legs, followed by the closure of
// Eq. 3.6.  Spans [a..b] are stored by length, then start.  The four-gluon sum is
// regrouped exactly: with S[x..y] = sum_k J[x..k].J[k+1..y] (the scalars the three-gluon
// sum already forms),
//   sum_{i<j} (JA.JB) JC = sum_j S[a..j] J[j+1..b],   sum_{i<j} (JC.JB) JA = sum_i S[i+1..b] J[a..i],
// so only 2 (JA.JC) JB is summed over pairs of splits.  Span momenta are never stored:
// every K[x..y] a bracket needs is summed left to right over its own legs in FP64 and only
// then cast to T (a difference of longer sums would lose relative precision on soft spans).
// K^2 and 1/K^2 are FP64, formed without fused multiply-adds, before the cast.
// ----------------------------------------------------------------------------------------
// K^2 of an FP64 four-vector, E^2 - px^2 - py^2 - pz^2 in that order, without contraction
__device__ __forceinline__ double minkowski_sq(const double K[4]) {
#pragma clang fp contract(off)
  const double e = K[0] * K[0];
  const double x = K[1] * K[1];
  const double y = K[2] * K[2];
  const double z = K[3] * K[3];
  return ((e - x) - y) - z;
}

// left-to-right FP64 sum of the legs A..B
template <int A, int B, int L>
__device__ __forceinline__ void span_sum(const double (&k)[L][4], double K[4]) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) K[mu] = k[A][mu];
  static_for<A + 1, B + 1>([&](auto i) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) K[mu] += k[decltype(i)::value][mu];
  });
}

// An optimisation barrier on a register value (no code is emitted): after it the compiler
// knows nothing of x, so it neither merges a computation that starts from x with another nor
// keeps what produced x live for later uses.
template <typename T>
__device__ __forceinline__ void opaque(T& x) {
  asm volatile("" : "+v"(x));
}

template <int L>
struct Spans {
  static constexpr int count = L * (L + 1) / 2;
  __host__ __device__ static constexpr int at(int a, int b) {
    return (b - a) * (L + 1) - (b - a) * (b - a + 1) / 2 + a;
  }
};

// Span momenta for the brackets, K[A..B] cast to T and covariant (K_mu = g_mu K^mu, so that
// J.K is a plain sum of products: the spatial signs are folded into K once instead of into
// every product), and the propagators 1/K^2, from the FP64 leg momenta at every use (any
// precision, any workgroup size).
template <int L, typename T>
struct SpanKLegs {
  const double (&k)[L][4];
  template <int A, int B>
  __device__ __forceinline__ void K(T out[4]) const {
    double d[4];
    span_sum<A, B, L>(k, d);
    out[0] = T(d[0]);
#pragma unroll
    for (int mu = 1; mu < 4; ++mu) out[mu] = T(-d[mu]);
  }
  template <int A, int B>
  __device__ __forceinline__ T prop() const {
    double d[4];
    span_sum<A, B, L>(k, d);
    return T(1.0 / minkowski_sq(d));
  }
};

// The same values from a per-lane table in LDS, filled once per event: every span momentum
// summed left to right in FP64 then cast to float (covariant), every propagator 1/K^2 formed
// in FP64.
// Layout [span][lane] with LANES lanes per workgroup, so a wave's accesses are contiguous.
template <int L, int LANES>
struct SpanKLds {
  float4* kt;  // &table[0][lane]
  float* pt;   // &props[0][lane]
  __device__ __forceinline__ void fill(const double (&k)[L][4]) {
    using SP = Spans<L>;
    static_for<0, L>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      double acc[4] = {k[a][0], k[a][1], k[a][2], k[a][3]};
      kt[SP::at(a, a) * LANES] = make_float4(float(acc[0]), float(-acc[1]), float(-acc[2]), float(-acc[3]));
      static_for<a + 1, L>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) acc[mu] += k[b][mu];
        kt[SP::at(a, b) * LANES] = make_float4(float(acc[0]), float(-acc[1]), float(-acc[2]), float(-acc[3]));
        // K^2 in FP64, its reciprocal in FP32 (within 1 ulp of the rounded K^2's)
        if (b - a + 1 < L) pt[SP::at(a, b) * LANES] = __builtin_amdgcn_rcpf(float(minkowski_sq(acc)));
      });
    });
  }
  template <int A, int B>
  __device__ __forceinline__ void K(float out[4]) const {
    const float4 v = kt[Spans<L>::at(A, B) * LANES];
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  }
  template <int A, int B>
  __device__ __forceinline__ float prop() const {
    return pt[Spans<L>::at(A, B) * LANES];
  }
};

// Fused multiply-add a * b + c with one rounding, in the precision of the operands.  The
// complex products below are written as chains of these (one accumulator per real part),
// which halves the separate adds a contracted a*b - c*d form would leave.
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// r + i i = x . y, bilinear with the metric (+,-,-,-)
template <typename T>
__device__ __forceinline__ void cdot(const cv4<T>& x, const cv4<T>& y, T& r, T& i) {
  r = fmac(-x.im[0], y.im[0], x.re[0] * y.re[0]);
  i = fmac(x.im[0], y.re[0], x.re[0] * y.im[0]);
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    r = fmac(-x.re[mu], y.re[mu], r);
    r = fmac(x.im[mu], y.im[mu], r);
    i = fmac(-x.re[mu], y.im[mu], i);
    i = fmac(-x.im[mu], y.re[mu], i);
  }
}

// r + i i = x . k for a real four-vector k given covariant (k_mu = g_mu k^mu)
template <typename T>
__device__ __forceinline__ void rdot(const cv4<T>& x, const T k[4], T& r, T& i) {
  r = x.re[0] * k[0];
  i = x.im[0] * k[0];
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    r = fmac(x.re[mu], k[mu], r);
    i = fmac(x.im[mu], k[mu], i);
  }
}

// K_A - K_B contravariant, from covariant K_A, K_B (exact: only signs differ)
template <typename T>
__device__ __forceinline__ T kdiff(const T (&ka)[4], const T (&kb)[4], int mu) {
  return mu == 0 ? ka[0] - kb[0] : kb[mu] - ka[mu];
}

// The same dot with its imaginary part returned negated (ni = -i, exactly: every step is the
// negation of cdot's), for products whose consumer then needs no negated operand.
template <typename T>
__device__ __forceinline__ void cdot_ni(const cv4<T>& x, const cv4<T>& y, T& r, T& ni) {
  r = fmac(-x.im[0], y.im[0], x.re[0] * y.re[0]);
  ni = fmac(-x.im[0], y.re[0], -x.re[0] * y.im[0]);
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    r = fmac(-x.re[mu], y.re[mu], r);
    r = fmac(x.im[mu], y.im[mu], r);
    ni = fmac(x.re[mu], y.im[mu], ni);
    ni = fmac(x.im[mu], y.re[mu], ni);
  }
}

// x . k with k covariant, its real part returned negated (nr = -r, exactly)
template <typename T>
__device__ __forceinline__ void rdot_nr(const cv4<T>& x, const T k[4], T& nr, T& i) {
  nr = -x.re[0] * k[0];
  i = x.im[0] * k[0];
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    nr = fmac(-x.re[mu], k[mu], nr);
    i = fmac(x.im[mu], k[mu], i);
  }
}

// acc += (cr - i nci) * y, the conjugate-sign form of caxpy (same roundings as
// caxpy(cr, -nci, y, acc))
template <typename T>
__device__ __forceinline__ void caxpy_nci(T cr, T nci, const cv4<T>& y, cv4<T>& acc) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    acc.re[mu] = fmac(nci, y.im[mu], fmac(cr, y.re[mu], acc.re[mu]));
    acc.im[mu] = fmac(-nci, y.re[mu], fmac(cr, y.im[mu], acc.im[mu]));
  }
}

// acc += (cr + i ci) * y
template <typename T>
__device__ __forceinline__ void caxpy(T cr, T ci, const cv4<T>& y, cv4<T>& acc) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    acc.re[mu] = fmac(-ci, y.im[mu], fmac(cr, y.re[mu], acc.re[mu]));
    acc.im[mu] = fmac(ci, y.re[mu], fmac(cr, y.im[mu], acc.im[mu]));
  }
}

// One span [A..B] of the recursion: its bracket sum V (Eqs. 3.1-3.2, regrouped as above).
// The span scalars are carried negated (nS = -S, exactly), which turns the S terms'
// subtractions into plain multiply-adds; sr, si return -S of [A..B].
template <int L, int A, int B, typename T, typename KS>
__device__ __forceinline__ void span_vertex(const KS& ks, const cv4<T> (&J)[Spans<L>::count],
                                            const T (&Sr)[Spans<L>::count], const T (&Si)[Spans<L>::count],
                                            cv4<T>& V, T& sr, T& si) {
  // every multiply-add below is an explicit fmac: the sum rounds identically wherever the
  // recursion is inlined (the compiler contracts nothing on its own)
#pragma clang fp contract(off)
  using SP = Spans<L>;
  cv4<T> X, Y;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) X.re[mu] = X.im[mu] = Y.re[mu] = Y.im[mu] = T(0);
  sr = T(0);
  si = T(0);
  // three-gluon brackets [J[A..i], J[i+1..B]]
  static_for<A, B>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int PA = SP::at(A, i), PB = SP::at(i + 1, B);
    T ka[4], kb[4];
    ks.template K<A, i>(ka);
    ks.template K<i + 1, B>(kb);
    T dr, di, ar, ai, nbr, bi;
    cdot(J[PA], J[PB], dr, di);
    rdot(J[PA], kb, ar, ai);
    rdot_nr(J[PB], ka, nbr, bi);
    caxpy(ar, ai, J[PB], X);
    caxpy_nci(nbr, bi, J[PA], X);  // X -= (J[PB].K_A) J[PA]
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const T dk = kdiff(ka, kb, mu);
      Y.re[mu] = fmac(dr, dk, Y.re[mu]);
      Y.im[mu] = fmac(di, dk, Y.im[mu]);
    }
    sr -= dr;
    si -= di;
  });
  // four-gluon brackets: 2 (JA.JC) JB over pairs of splits
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<i + 1, B>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      T dr, ndi;
      cdot_ni(J[SP::at(A, i)], J[SP::at(j + 1, B)], dr, ndi);
      caxpy_nci(dr, ndi, J[SP::at(i + 1, j)], X);
    });
  });
  // -(JA.JB) JC and -(JC.JB) JA through the span scalars S
  static_for<A + 1, B>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    constexpr int Sx = SP::at(A, j);
    caxpy(Sr[Sx], Si[Sx], J[SP::at(j + 1, B)], Y);
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int Sx = SP::at(i + 1, B);
    caxpy(Sr[Sx], Si[Sx], J[SP::at(A, i)], Y);
  });
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    V.re[mu] = fmac(T(2), X.re[mu], Y.re[mu]);
    V.im[mu] = fmac(T(2), X.im[mu], Y.im[mu]);
  }
}

// Forward recursion: fills every stored current J and negated span scalar -S, and returns
// the undivided bracket sum V of the full span [0..L-1].
template <int L, typename T, typename KS>
__device__ __forceinline__ void bg_forward(const KS& ks, const cv4<T> (&src)[L],
                                           cv4<T> (&J)[Spans<L>::count], T (&Sr)[Spans<L>::count],
                                           T (&Si)[Spans<L>::count], cv4<T>& Vfull) {
  using SP = Spans<L>;
  static_for<0, L>([&](auto ac) { J[decltype(ac)::value] = src[decltype(ac)::value]; });
  static_for<2, L>([&](auto lc) {
    constexpr int len = decltype(lc)::value;
    static_for<0, L - len + 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value, b = a + len - 1, s = SP::at(a, b);
      cv4<T> V;
      T sr, si;
      span_vertex<L, a, b, T>(ks, J, Sr, Si, V, sr, si);
      const T prop = ks.template prop<a, b>();
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        J[s].re[mu] = V.re[mu] * prop;
        J[s].im[mu] = V.im[mu] * prop;
      }
      Sr[s] = sr;
      Si[s] = si;
    });
  });
  // the full span: amputated (Eq. 3.6), never divided by its vanishing K^2
  T sr, si;
  span_vertex<L, 0, L - 1, T>(ks, J, Sr, Si, Vfull, sr, si);
}

// k: FP64 all-outgoing momenta of the L recursion legs (any common power-of-two scale);
// src: their sources; eps0: the closing leg's polarisation.  Returns m = eps0 . V.
template <int L, typename T, typename KS>
__device__ __forceinline__ void bg_amplitude(const KS& ks, const cv4<T> (&src)[L], const cv4<T>& eps0,
                                             double& m_re, double& m_im) {
  using SP = Spans<L>;
  cv4<T> J[SP::count];
  T Sr[SP::count], Si[SP::count];
  cv4<T> V;
  bg_forward<L, T>(ks, src, J, Sr, Si, V);
  T mr, mi;
  cdot(eps0, V, mr, mi);
  m_re = double(mr);
  m_im = double(mi);
}

// ----------------------------------------------------------------------------------------
// Real currents (the paper's choice of sources, Sec. 3): every source is a real unit vector
// orthogonal to its momentum, eps = cos(psi) e1 + sin(psi) e2 with the transverse basis
// e1 = (0, cos t cos f, cos t sin f, -sin t), e2 = (0, -sin f, cos f, 0) of the physical
// momentum (the helicity vectors above are (-h e1 - i e2)/sqrt 2), psi uniform.  Then every
// current is real: the same brackets and closure as above with real four-vectors, a
// quarter of the multiplications and half of the storage.  2^n |A(eps)|^2 averages over
// the angles to the helicity sum.
// ----------------------------------------------------------------------------------------
template <typename T>
struct rv4 {
  T v[4];
};

// (cos psi, sin psi) as (c, s); no implicit fused multiply-adds, as polarisation()
template <typename T>
__device__ __forceinline__ rv4<T> real_polarisation(const double p[4], T c, T s) {
#pragma clang fp contract(off)
  const T px = T(p[1]), py = T(p[2]), pz = T(p[3]);
  const T pt2 = px * px + py * py;
  T ct, st, cf = T(1), sf = T(0);
  if constexpr (std::is_same<T, float>::value) {
    const float ipa = __builtin_amdgcn_rsqf(pt2 + pz * pz);
    const float ipt = __builtin_amdgcn_rsqf(pt2);
    ct = pz * ipa;
    st = pt2 > 0.0f ? (pt2 * ipt) * ipa : 0.0f;
    if (pt2 > 0.0f) {
      cf = px * ipt;
      sf = py * ipt;
    }
  } else {
    const T pa = sqrt(pt2 + pz * pz);
    const T pt = sqrt(pt2);
    const T ipa = T(1) / pa;
    ct = pz * ipa;
    st = pt * ipa;
    if (pt2 > T(0)) {
      const T ipt = T(1) / pt;
      cf = px * ipt;
      sf = py * ipt;
    }
  }
  rv4<T> e;
  e.v[0] = T(0);
  e.v[1] = fmac(c * ct, cf, -(s * sf));
  e.v[2] = fmac(c * ct, sf, s * cf);
  e.v[3] = -(c * st);
  return e;
}

// x . y (metric (+,-,-,-)) of real four-vectors
template <typename T>
__device__ __forceinline__ T vdot(const rv4<T>& x, const rv4<T>& y) {
  T r = x.v[0] * y.v[0];
  r = fmac(-x.v[1], y.v[1], r);
  r = fmac(-x.v[2], y.v[2], r);
  return fmac(-x.v[3], y.v[3], r);
}

// x . k for k given covariant
template <typename T>
__device__ __forceinline__ T vdot_cov(const rv4<T>& x, const T (&k)[4]) {
  T r = x.v[0] * k[0];
  r = fmac(x.v[1], k[1], r);
  r = fmac(x.v[2], k[2], r);
  return fmac(x.v[3], k[3], r);
}

// acc += c y
template <typename T>
__device__ __forceinline__ void vaxpy(T c, const rv4<T>& y, rv4<T>& acc) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) acc.v[mu] = fmac(c, y.v[mu], acc.v[mu]);
}

// One span [A..B] with real currents: its bracket sum V (regrouped as span_vertex; span
// scalars negated as there).
template <int L, int A, int B, typename T, typename KS>
__device__ __forceinline__ void span_vertex_r(const KS& ks, const rv4<T> (&J)[Spans<L>::count],
                                              const T (&S)[Spans<L>::count], rv4<T>& V, T& sv) {
#pragma clang fp contract(off)
  using SP = Spans<L>;
  rv4<T> X, Y;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) X.v[mu] = Y.v[mu] = T(0);
  sv = T(0);
  static_for<A, B>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int PA = SP::at(A, i), PB = SP::at(i + 1, B);
    T ka[4], kb[4];
    ks.template K<A, i>(ka);
    ks.template K<i + 1, B>(kb);
    const T d = vdot(J[PA], J[PB]);
    vaxpy(vdot_cov(J[PA], kb), J[PB], X);
    vaxpy(-vdot_cov(J[PB], ka), J[PA], X);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) Y.v[mu] = fmac(d, kdiff(ka, kb, mu), Y.v[mu]);
    sv -= d;
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<i + 1, B>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      vaxpy(vdot(J[SP::at(A, i)], J[SP::at(j + 1, B)]), J[SP::at(i + 1, j)], X);
    });
  });
  static_for<A + 1, B>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    vaxpy(S[SP::at(A, j)], J[SP::at(j + 1, B)], Y);
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    vaxpy(S[SP::at(i + 1, B)], J[SP::at(A, i)], Y);
  });
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) V.v[mu] = fmac(T(2), X.v[mu], Y.v[mu]);
}

// Real recursion and closure m = eps0 . V[0..L-1].
template <int L, typename T, typename KS>
__device__ __forceinline__ double bg_amplitude_r(const KS& ks, const rv4<T> (&src)[L], const rv4<T>& eps0) {
  using SP = Spans<L>;
  rv4<T> J[SP::count];
  T S[SP::count];
  static_for<0, L>([&](auto ac) { J[decltype(ac)::value] = src[decltype(ac)::value]; });
  static_for<2, L>([&](auto lc) {
    constexpr int len = decltype(lc)::value;
    static_for<0, L - len + 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value, b = a + len - 1, s = SP::at(a, b);
      rv4<T> V;
      T sv;
      span_vertex_r<L, a, b, T>(ks, J, S, V, sv);
      const T prop = ks.template prop<a, b>();
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) J[s].v[mu] = V.v[mu] * prop;
      S[s] = sv;
    });
  });
  rv4<T> V;
  T sv;
  span_vertex_r<L, 0, L - 1, T>(ks, J, S, V, sv);
  return double(vdot(eps0, V));
}

// ----------------------------------------------------------------------------------------
// Compensated sums: TwoSum (Knuth) pairs (s, c).
// ----------------------------------------------------------------------------------------
struct CSum {
  double s, c;
};

__device__ __forceinline__ CSum cs_add(CSum x, CSum y) {
  const double s = x.s + y.s;
  const double bb = s - x.s;
  const double e = (x.s - (s - bb)) + (y.s - bb);
  return CSum{s, x.c + y.c + e};
}

}  // namespace bgk
