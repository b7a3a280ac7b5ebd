// Hand-written adjoint of the event path: d log w_int / d(RAMBO uniforms, x1, x2).
//
// log w_int = a log x1 + b log(1-x1) + a log x2 + b log(1-x2) + (n-5) log s_hat + log|A|^2 + c
// (the integrand of Eq. 3.8 without the cut step function and without the sampling density;
// the flux 1/s_hat and RAMBO's volume s_hat^(n-4) give the s_hat power).  |A|^2 is evaluated on
// the partonic centre-of-mass momenta, so the reverse sweep runs: closure -> recursion
// (Eqs. 3.1-3.2, regrouped as in the forward) -> helicity sources -> momenta -> RAMBO's
// conformal map -> q(rho) -> uniforms, and sqrt(s_hat) -> x1, x2.  The forward is recomputed
// in the kernel; no current is kept between the two calls of the torch Function.
//
// Complex adjoints are carried as zb = dL/dRe z + i dL/dIm z, so for a bilinear w = x y the
// rule is xb += conj(y) wb, and a real factor r of a complex z gets rb += Re(conj(z) wb).
#pragma once

#include "bg_group_adj.hpp"
#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

template <typename T>
__device__ __forceinline__ T gsign(int mu) {
  return mu == 0 ? T(1) : T(-1);
}

// r + i i = x . k for a contravariant real four-vector k (the reverse sweep keeps its span
// momenta contravariant)
template <typename T>
__device__ __forceinline__ void rdot_contra(const cv4<T>& x, const T k[4], T& r, T& i) {
  r = x.re[0] * k[0];
  i = x.im[0] * k[0];
#pragma unroll
  for (int mu = 1; mu < 4; ++mu) {
    r = fmac(-x.re[mu], k[mu], r);
    i = fmac(-x.im[mu], k[mu], i);
  }
}

// from d = x.y (bilinear Minkowski): xb_mu += g_mu conj(y_mu) db
template <typename T>
__device__ __forceinline__ void cdot_adj(const cv4<T>& y, T dbr, T dbi, cv4<T>& xb) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const T g = gsign<T>(mu);
    xb.re[mu] = fmac(g * y.im[mu], dbi, fmac(g * y.re[mu], dbr, xb.re[mu]));
    xb.im[mu] = fmac(-g * y.im[mu], dbr, fmac(g * y.re[mu], dbi, xb.im[mu]));
  }
}

// from acc += c y (complex c): yb += conj(c) accb
template <typename T>
__device__ __forceinline__ void caxpy_adj_y(T cr, T ci, const cv4<T>& accb, cv4<T>& yb) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    yb.re[mu] = fmac(ci, accb.im[mu], fmac(cr, accb.re[mu], yb.re[mu]));
    yb.im[mu] = fmac(-ci, accb.re[mu], fmac(cr, accb.im[mu], yb.im[mu]));
  }
}

// from acc += c y: cb += sum_mu conj(y_mu) accb_mu
template <typename T>
__device__ __forceinline__ void caxpy_adj_c(const cv4<T>& y, const cv4<T>& accb, T& cbr, T& cbi) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    cbr = fmac(y.im[mu], accb.im[mu], fmac(y.re[mu], accb.re[mu], cbr));
    cbi = fmac(-y.im[mu], accb.re[mu], fmac(y.re[mu], accb.im[mu], cbi));
  }
}

// add a span-momentum adjoint to each of the legs A..B
template <int A, int B, int L, typename T>
__device__ __forceinline__ void spread(const T Kb[4], T (&kb)[L][4]) {
  static_for<A, B + 1>([&](auto tc) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) kb[decltype(tc)::value][mu] += Kb[mu];
  });
}

// Reverse of span_vertex for span [A..B]: given Vb (adjoint of its bracket sum V) and the
// adjoint (sbr, sbi) of its scalar S, accumulate into the adjoints of the sub-currents,
// sub-span scalars and leg momenta.
template <int L, int A, int B, typename T>
__device__ __forceinline__ void span_vertex_adj(const double (&k)[L][4], const cv4<T> (&J)[Spans<L>::count],
                                                const T (&Sr)[Spans<L>::count], const T (&Si)[Spans<L>::count],
                                                const cv4<T>& Vb, T sbr, T sbi, cv4<T> (&Jb)[Spans<L>::count],
                                                T (&Sbr)[Spans<L>::count], T (&Sbi)[Spans<L>::count],
                                                T (&kb)[L][4]) {
  using SP = Spans<L>;
  // V = 2X + Y
  cv4<T> Xb, Yb;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Xb.re[mu] = T(2) * Vb.re[mu];
    Xb.im[mu] = T(2) * Vb.im[mu];
    Yb.re[mu] = Vb.re[mu];
    Yb.im[mu] = Vb.im[mu];
  }
  // Y -= S[A..j] J[j+1..B]  and  Y -= S[i+1..B] J[A..i]
  static_for<A + 1, B>([&](auto jc) {
    constexpr int j = decltype(jc)::value, Sx = SP::at(A, j), Jx = SP::at(j + 1, B);
    T cr = T(0), ci = T(0);
    caxpy_adj_c(J[Jx], Yb, cr, ci);
    Sbr[Sx] -= cr;
    Sbi[Sx] -= ci;
    caxpy_adj_y(-Sr[Sx], -Si[Sx], Yb, Jb[Jx]);
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value, Sx = SP::at(i + 1, B), Jx = SP::at(A, i);
    T cr = T(0), ci = T(0);
    caxpy_adj_c(J[Jx], Yb, cr, ci);
    Sbr[Sx] -= cr;
    Sbi[Sx] -= ci;
    caxpy_adj_y(-Sr[Sx], -Si[Sx], Yb, Jb[Jx]);
  });
  // X += (J[A..i] . J[j+1..B]) J[i+1..j]
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<i + 1, B>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int PA = SP::at(A, i), PM = SP::at(i + 1, j), PC = SP::at(j + 1, B);
      T er, ei;
      cdot(J[PA], J[PC], er, ei);
      T ebr = T(0), ebi = T(0);
      caxpy_adj_c(J[PM], Xb, ebr, ebi);
      caxpy_adj_y(er, ei, Xb, Jb[PM]);
      cdot_adj(J[PC], ebr, ebi, Jb[PA]);
      cdot_adj(J[PA], ebr, ebi, Jb[PC]);
    });
  });
  // three-gluon brackets
  static_for<A, B>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int PA = SP::at(A, i), PB = SP::at(i + 1, B);
    double KAd[4], KBd[4];
    span_sum<A, i, L>(k, KAd);
    span_sum<i + 1, B, L>(k, KBd);
    T ka[4], kbv[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      ka[mu] = T(KAd[mu]);
      kbv[mu] = T(KBd[mu]);
    }
    T dr, di, ar, ai, br, bi;
    cdot(J[PA], J[PB], dr, di);
    rdot_contra(J[PA], kbv, ar, ai);
    rdot_contra(J[PB], ka, br, bi);
    // X += ca J[PB] - cb J[PA]
    T cabr = T(0), cabi = T(0), cbbr = T(0), cbbi = T(0);
    caxpy_adj_c(J[PB], Xb, cabr, cabi);
    caxpy_adj_y(ar, ai, Xb, Jb[PB]);
    caxpy_adj_c(J[PA], Xb, cbbr, cbbi);
    cbbr = -cbbr;
    cbbi = -cbbi;
    caxpy_adj_y(-br, -bi, Xb, Jb[PA]);
    // Y += d (KA - KB);  S += d
    T dbr = sbr, dbi = sbi;
    T KAb[4], KBb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const T dk = ka[mu] - kbv[mu];
      dbr += dk * Yb.re[mu];
      dbi += dk * Yb.im[mu];
      const T w = dr * Yb.re[mu] + di * Yb.im[mu];  // Re(conj(d) Yb_mu)
      KAb[mu] = w;
      KBb[mu] = -w;
    }
    // d = J[PA] . J[PB]
    cdot_adj(J[PB], dbr, dbi, Jb[PA]);
    cdot_adj(J[PA], dbr, dbi, Jb[PB]);
    // ca = J[PA] . KB,  cb = J[PB] . KA
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const T g = gsign<T>(mu);
      Jb[PA].re[mu] += g * kbv[mu] * cabr;
      Jb[PA].im[mu] += g * kbv[mu] * cabi;
      KBb[mu] += g * (J[PA].re[mu] * cabr + J[PA].im[mu] * cabi);
      Jb[PB].re[mu] += g * ka[mu] * cbbr;
      Jb[PB].im[mu] += g * ka[mu] * cbbi;
      KAb[mu] += g * (J[PB].re[mu] * cbbr + J[PB].im[mu] * cbbi);
    }
    spread<A, i, L, T>(KAb, kb);
    spread<i + 1, B, L, T>(KBb, kb);
  });
}

// Reverse sweep of bg_forward + closure.  mb: adjoint of m = eps0 . V.  Outputs the adjoints
// of the sources (srcb), of the closing polarisation (e0b) and of the scaled leg momenta (kb).
template <int L, typename T>
__device__ __forceinline__ void bg_reverse(const double (&k)[L][4], const cv4<T> (&J)[Spans<L>::count],
                                           const T (&Sr)[Spans<L>::count], const T (&Si)[Spans<L>::count],
                                           const cv4<T>& eps0, const cv4<T>& Vfull, T mbr, T mbi,
                                           cv4<T> (&srcb)[L], cv4<T>& e0b, T (&kb)[L][4]) {
  using SP = Spans<L>;
  cv4<T> Jb[SP::count];
  T Sbr[SP::count], Sbi[SP::count];
  static_for<0, SP::count>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) Jb[s].re[mu] = Jb[s].im[mu] = T(0);
    Sbr[s] = Sbi[s] = T(0);
  });
  static_for<0, L>([&](auto tc) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) kb[decltype(tc)::value][mu] = T(0);
  });
  // m = eps0 . V
  cv4<T> Vb;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) Vb.re[mu] = Vb.im[mu] = e0b.re[mu] = e0b.im[mu] = T(0);
  cdot_adj(eps0, mbr, mbi, Vb);
  cdot_adj(Vfull, mbr, mbi, e0b);
  span_vertex_adj<L, 0, L - 1, T>(k, J, Sr, Si, Vb, T(0), T(0), Jb, Sbr, Sbi, kb);
  // lengths L-1 down to 2
  static_for<0, L - 2>([&](auto rc) {
    constexpr int len = L - 1 - decltype(rc)::value;
    static_for<0, L - len + 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value, b = a + len - 1, s = SP::at(a, b);
      double Kd[4];
      span_sum<a, b, L>(k, Kd);
      const T prop = T(1.0 / minkowski_sq(Kd));
      // J = V prop:  Vb = prop Jb;  K_mu gets -2 g_mu K_mu prop sum Re(conj(J) Jb)
      cv4<T> Vbs;
      T rj = T(0);
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        Vbs.re[mu] = prop * Jb[s].re[mu];
        Vbs.im[mu] = prop * Jb[s].im[mu];
        rj += J[s].re[mu] * Jb[s].re[mu] + J[s].im[mu] * Jb[s].im[mu];
      }
      T Kb[4];
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) Kb[mu] = T(-2) * gsign<T>(mu) * T(Kd[mu]) * prop * rj;
      spread<a, b, L, T>(Kb, kb);
      span_vertex_adj<L, a, b, T>(k, J, Sr, Si, Vbs, Sbr[s], Sbi[s], Jb, Sbr, Sbi, kb);
    });
  });
  static_for<0, L>([&](auto tc) { srcb[decltype(tc)::value] = Jb[decltype(tc)::value]; });
}

// Adjoint of polarisation(): accumulates dL/dp (spatial components) from eb.
template <typename T>
__device__ __forceinline__ void polarisation_adj(const double p[4], bool plus, const cv4<T>& eb, double pb[4]) {
  const double px = p[1], py = p[2], pz = p[3];
  const double pt2 = px * px + py * py;
  if (!(pt2 > 0.0)) return;  // a leg along the beam axis: its direction is fixed
  const double pa = sqrt(pt2 + pz * pz), pt = sqrt(pt2);
  const double ct = pz / pa, cf = px / pt, sf = py / pt;
  const double r = 0.70710678118654752440;
  const double hs = plus ? 1.0 : -1.0;
  const double e1r = double(eb.re[1]), e1i = double(eb.im[1]);
  const double e2r = double(eb.re[2]), e2i = double(eb.im[2]);
  const double e3r = double(eb.re[3]);
  const double ctb = -hs * r * (cf * e1r + sf * e2r);
  const double stb = hs * r * e3r;
  const double cfb = -hs * r * ct * e1r - r * e2i;
  const double sfb = r * e1i - hs * r * ct * e2r;
  const double pa3 = pa * pa * pa, pt3 = pt2 * pt;
  pb[1] += ctb * (-pz * px / pa3) + stb * (px * pz * pz / (pt * pa3)) + cfb * (py * py / pt3) + sfb * (-px * py / pt3);
  pb[2] += ctb * (-pz * py / pa3) + stb * (py * pz * pz / (pt * pa3)) + cfb * (-px * py / pt3) + sfb * (px * px / pt3);
  pb[3] += ctb * (pt2 / pa3) + stb * (-pt * pz / pa3);
}

struct RamboMapAdj {
  double bxb, byb, bzb, gammab, ab, Xb;
};

// Adjoint of RamboMap::apply for one particle.
__device__ __forceinline__ void rambo_apply_adj(const RamboMap& m, const double q[4], const double pb[4], double qb[4],
                                                RamboMapAdj& A) {
  const double b[3] = {m.bx, m.by, m.bz};
  const double bq = b[0] * q[1] + b[1] * q[2] + b[2] * q[3];
  double inner = m.gamma * q[0] + bq;
  A.Xb += pb[0] * inner;
  const double e = m.X * pb[0];
  A.gammab += e * q[0];
  qb[0] += e * m.gamma;
  double bqb = e;
  double bb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    inner = q[j + 1] + b[j] * q[0] + m.a * bq * b[j];
    A.Xb += pb[j + 1] * inner;
    const double P = m.X * pb[j + 1];
    qb[j + 1] += P;
    bb[j] += P * q[0] + P * m.a * bq;
    qb[0] += P * b[j];
    A.ab += P * bq * b[j];
    bqb += P * m.a * b[j];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    bb[j] += bqb * q[j + 1];
    qb[j + 1] += bqb * b[j];
  }
  A.bxb += bb[0];
  A.byb += bb[1];
  A.bzb += bb[2];
}

// Adjoint of RamboMap::init: accumulates dL/dQ and dL/dsqrt(s_hat).
__device__ __forceinline__ void rambo_init_adj(const RamboMap& m, const double Q[4], const RamboMapAdj& A,
                                               double Qb[4], double& sb) {
  const double Mv = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  sb += A.Xb / Mv;
  double Mb = -A.Xb * m.X / Mv;
  const double gammab = A.gammab - A.ab * m.a * m.a;
  Qb[0] += gammab / Mv;
  Mb += -gammab * m.gamma / Mv;
  const double b[3] = {m.bx, m.by, m.bz};
  const double bb[3] = {A.bxb, A.byb, A.bzb};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Qb[j + 1] += -bb[j] / Mv;
    Mb += -bb[j] * b[j] / Mv;
  }
  const double M2b = Mb / (2.0 * Mv);
  Qb[0] += 2.0 * Q[0] * M2b;
#pragma unroll
  for (int j = 0; j < 3; ++j) Qb[j + 1] += -2.0 * Q[j + 1] * M2b;
}

// Adjoint of rambo_q: rho adjoints from q adjoints.
__device__ __forceinline__ void rambo_q_adj(double r1, double r2, double r3, double r4, const double qb[4],
                                            double rb[4]) {
  const double c = 2.0 * r1 - 1.0;
  const double st = sqrt(1.0 - c * c);
  double sp, cp;
  sincospi_fp64(2.0 * r2, &sp, &cp);
  const double q0 = -log_fp64(r3 * r4);
  const double q0b = qb[0] + qb[1] * st * cp + qb[2] * st * sp + qb[3] * c;
  const double stb = q0 * (qb[1] * cp + qb[2] * sp);
  const double cpb = q0 * st * qb[1], spb = q0 * st * qb[2];
  const double cb = q0 * qb[3] - stb * c / st;
  rb[0] = 2.0 * cb;
  rb[1] = 2.0 * 3.14159265358979323846 * (cp * spb - sp * cpb);
  rb[2] = -q0b / r3;
  rb[3] = -q0b / r4;
}

// Per-event kinematics of the gradient kernels (partonic centre-of-mass frame).
template <int N>
struct GradKin {
  uint32_t leg[N];
  uint32_t hel;
  double x1, x2, shat, rs;
  double q[N][4];   // RAMBO's q (position order; beam positions unused)
  double Q[4];
  RamboMap map;
  double pc[N][4];  // physical CM momenta, position order
  int ex;           // momentum scale 2^-ex of the recursion
  double sc;
};

template <int N>
__device__ __forceinline__ void grad_front(const GradArgs& G, int64_t i, GradKin<N>& K) {
  constexpr int NF = N - 2;
  K.leg[0] = 0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const uint32_t l = G.order[i * N + t];
    K.leg[t] = l < 1u ? 1u : (l > (uint32_t)(N - 1) ? (uint32_t)(N - 1) : l);
  }
  K.hel = G.hel[i];
  K.x1 = 1.0;
  K.x2 = 1.0;
  K.shat = G.sqrt_s * G.sqrt_s;
  K.rs = G.sqrt_s;
  if (G.use_pdf) {
    K.x1 = G.x12[2 * i];
    K.x2 = G.x12[2 * i + 1];
    K.shat = K.x1 * K.x2 * G.sqrt_s * G.sqrt_s;
    K.rs = sqrt(K.shat);
  }
  // RAMBO in position order (centre-of-mass frame)
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) K.Q[mu] = 0.0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const bool out = K.leg[t] >= 2u;
    const uint32_t pidx = out ? K.leg[t] - 2u : 0u;
    const double* u = G.u + (i * NF + pidx) * 4;
    rambo_q(u[0], u[1], u[2], u[3], K.q[t]);
    if (out) {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) K.Q[mu] += K.q[t][mu];
    }
  }
  K.map.init(K.Q, K.rs);
#pragma unroll
  for (int t = 0; t < N; ++t) {
    K.map.apply(K.q[t], K.pc[t]);
    if (K.leg[t] < 2u) {
      const double zs = K.leg[t] == 0u ? 0.5 * K.rs : -0.5 * K.rs;
      K.pc[t][0] = 0.5 * K.rs; K.pc[t][1] = 0.0; K.pc[t][2] = 0.0; K.pc[t][3] = zs;
    }
  }
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) esum += fabs(K.pc[t][0]);
  K.ex = ilogb(0.5 * esum);
  K.sc = ldexp(1.0, -K.ex);
}

// log w_int from |m|^2 of the scaled momenta; false (and zero gradients written) when
// |m|^2 vanishes or is not finite.
template <int N>
__device__ __forceinline__ bool grad_logw(const GradArgs& G, int64_t i, const GradKin<N>& K, double m2, bool store) {
  constexpr int NF = N - 2;
  const double ln2 = 0.69314718055994530942;
  double lw = log(m2) + (double)(2 * K.ex * (4 - N) - (N - 2)) * ln2 + (N - 5) * log(K.shat) + G.log_const;
  if (G.use_pdf) lw += G.pdf_a * (log(K.x1) + log(K.x2)) + G.pdf_b * (log1p(-K.x1) + log1p(-K.x2));
  if (!(m2 > 0.0) || !isfinite(m2)) {
    if (store) {
      double* gu = G.grad_u + i * NF * 4;
      for (int c = 0; c < NF * 4; ++c) gu[c] = 0.0;
      G.grad_x[2 * i] = 0.0;
      G.grad_x[2 * i + 1] = 0.0;
      if (G.logw) G.logw[i] = -INFINITY;
    }
    return false;
  }
  if (store && G.logw) G.logw[i] = lw;
  return true;
}

// From the CM momentum adjoints pb (polarisation adjoints included) and the sqrt(s_hat)
// adjoint of the beams: RAMBO's conformal map, q(rho), and x1, x2; writes the gradients.
template <int N>
__device__ __forceinline__ void grad_back(const GradArgs& G, int64_t i, const GradKin<N>& K, const double (&pb)[N][4],
                                          double rsb) {
  constexpr int NF = N - 2;
  const double gw = G.gout ? G.gout[i] : 1.0;
  RamboMapAdj A{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double qb[N][4];
#pragma unroll
  for (int t = 1; t < N; ++t) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) qb[t][mu] = 0.0;
    if (K.leg[t] >= 2u) rambo_apply_adj(K.map, K.q[t], pb[t], qb[t], A);
  }
  double Qb[4] = {0.0, 0.0, 0.0, 0.0};
  rambo_init_adj(K.map, K.Q, A, Qb, rsb);
  double* gu = G.grad_u + i * NF * 4;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    if (K.leg[t] >= 2u) {
      const uint32_t pidx = K.leg[t] - 2u;
      const double* u = G.u + (i * NF + pidx) * 4;
      double qbt[4], rb[4];
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) qbt[mu] = qb[t][mu] + Qb[mu];
      rambo_q_adj(u[0], u[1], u[2], u[3], qbt, rb);
      double* o = gu + pidx * 4;
      o[0] = gw * rb[0]; o[1] = gw * rb[1]; o[2] = gw * rb[2]; o[3] = gw * rb[3];
    }
  }
  // s_hat = x1 x2 S:  d sqrt(s_hat) / dx_i = sqrt(s_hat) / (2 x_i)
  double xb1 = 0.0, xb2 = 0.0;
  if (G.use_pdf) {
    xb1 = rsb * K.rs / (2.0 * K.x1) + (N - 5) / K.x1 + G.pdf_a / K.x1 - G.pdf_b / (1.0 - K.x1);
    xb2 = rsb * K.rs / (2.0 * K.x2) + (N - 5) / K.x2 + G.pdf_a / K.x2 - G.pdf_b / (1.0 - K.x2);
  }
  G.grad_x[2 * i] = gw * xb1;
  G.grad_x[2 * i + 1] = gw * xb2;
}

// The recursion's adjoints go to the second kernel (k_grad_back), which takes them through
// the helicity sources, the momentum scaling, RAMBO and x1, x2: kept in one kernel, those
// values stay live across the reverse sweep and spill to scratch.  Per position t = 1..N-1
// twelve words: the contravariant adjoint of the scaled recursion momentum (4), then the
// source adjoint's real (4) and imaginary (4) parts; then a flag (0: |A|^2 = 0, nothing to
// do).  Layout [word][event], so neighbouring lanes write neighbouring words.
template <int N>
struct GradRaw {
  static constexpr int words = 12 * (N - 1) + 1;
  __host__ __device__ static constexpr int at(int t, int w) { return 12 * (t - 1) + w; }
};

// One event per lane: forward (CM momenta, recursion), log w_int, reverse sweep, momentum
// adjoints.
template <int N, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_grad(GradArgs G) {
  constexpr int L = N - 1;
  using SP = Spans<L>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.count) return;
  GradKin<N> K;
  grad_front<N>(G, i, K);
  double k[L][4];
  cv4<T> src[L];
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = K.leg[t] < 2u ? -K.sc : K.sc;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) k[t - 1][mu] = sg * K.pc[t][mu];
    src[t - 1] = polarisation<T>(K.pc[t], (K.hel >> K.leg[t]) & 1u);
  }
  const cv4<T> e0 = polarisation<T>(K.pc[0], K.hel & 1u);
  cv4<T> J[SP::count];
  T Sr[SP::count], Si[SP::count];
  cv4<T> V;
  SpanKLegs<L, T> ks{k};
  bg_forward<L, T>(ks, src, J, Sr, Si, V);
  // bg_forward leaves the span scalars negated; the reverse sweep takes S itself
  static_for<L, SP::count>([&](auto sc) {
    Sr[decltype(sc)::value] = -Sr[decltype(sc)::value];
    Si[decltype(sc)::value] = -Si[decltype(sc)::value];
  });
  T mr, mi;
  cdot(e0, V, mr, mi);
  const double m2 = double(mr) * double(mr) + double(mi) * double(mi);
  if (!grad_logw<N>(G, i, K, m2, true)) {
    G.pbuf[(GradRaw<N>::words - 1) * G.count + i] = 0.0;  // nothing for the second kernel
    return;
  }
  // reverse sweep: d log|m|^2 / dm = 2 m / |m|^2
  cv4<T> srcb[L], e0b;
  T kb[L][4];
  bg_reverse<L, T>(k, J, Sr, Si, e0, V, T(2.0 * double(mr) / m2), T(2.0 * double(mi) / m2), srcb, e0b, kb);
  double* o = G.pbuf + i;
#pragma unroll
  for (int t = 1; t < N; ++t) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      o[GradRaw<N>::at(t, mu) * G.count] = double(kb[t - 1][mu]);
      o[GradRaw<N>::at(t, 4 + mu) * G.count] = double(srcb[t - 1].re[mu]);
      o[GradRaw<N>::at(t, 8 + mu) * G.count] = double(srcb[t - 1].im[mu]);
    }
  }
  o[(GradRaw<N>::words - 1) * G.count] = 1.0;
}

// Whether the gradient kernel keeps its span scalars distributed over the lanes of a group:
// it holds the currents and their adjoints (twice the forward's registers).
template <int L, int G, typename T>
constexpr bool grad_dist_scalars() {
  return G > 1 && Spans<L>::count * 4 * (4 / G) * (int)(sizeof(T) / 4) > 160;
}

// GL lanes per event (the grouped recursion and its reverse sweep, bg_group_adj.hpp); every
// lane evaluates the kinematics, lane g writes its components of the raw adjoints.  The
// forward values pass an optimisation barrier before the sweep, so the compiler does not keep
// the forward pass's intermediates live across it.  Workgroups of 256 lanes.
template <int N, typename T, int GL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_grad_g(GradArgs G) {
  constexpr int L = N - 1, C = 4 / GL;
  using SP = Spans<L>;
  using SS = SpanScalars<L, GL, T, grad_dist_scalars<L, GL, T>()>;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GL;
  const int g = (int)(threadIdx.x % GL);
  if (i >= G.count) return;
  GradKin<N> K;
  grad_front<N>(G, i, K);
  const LaneShare<GL, T> ls(g);
  const LaneShare<GL, double> lsd(g);
  double k[L][C];  // covariant, this lane's components
  cvl<T, C> src[L], e0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = K.leg[t] < 2u ? -K.sc : K.sc;
#pragma unroll
    for (int c = 0; c < C; ++c) k[t - 1][c] = lsd.sg[c] * (sg * lsd.template pick<true>(K.pc[t], c));
    const cv4<T> e = polarisation<T>(K.pc[t], (K.hel >> K.leg[t]) & 1u);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      src[t - 1].re[c] = ls.template pick<true>(e.re, c);
      src[t - 1].im[c] = ls.template pick<true>(e.im, c);
    }
  }
  {
    const cv4<T> e = polarisation<T>(K.pc[0], K.hel & 1u);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      e0.re[c] = ls.template pick<true>(e.re, c);
      e0.im[c] = ls.template pick<true>(e.im, c);
    }
  }
  SpanKGroup<L, GL, T, true> ks{k, lsd.sg};
  cvl<T, C> J[SP::count];
  SS S(g);
  cvl<T, C> V;
  bg_forward_g<L, GL, T>(ls, ks, src, J, S, V);
  T mr, mi;
  cdot_g<GL>(ls, e0, V, mr, mi);
  const double m2 = double(mr) * double(mr) + double(mi) * double(mi);
  if (!grad_logw<N>(G, i, K, m2, g == 0)) {
    if (g == 0) G.pbuf[(GradRaw<N>::words - 1) * G.count + i] = 0.0;  // nothing for the second kernel
    return;
  }
  static_for<0, SP::count>([&](auto sc) {
    constexpr int q = decltype(sc)::value;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      opaque(J[q].re[c]);
      opaque(J[q].im[c]);
    }
  });
#pragma unroll
  for (int m = 0; m < SS::kSlots; ++m) {
    opaque(S.re[m]);
    opaque(S.im[m]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    opaque(V.re[c]);
    opaque(V.im[c]);
  }
  cvl<T, C> srcb[L], e0b;
  T kb[L][C];
  bg_reverse_g<L, GL, T>(ls, ks, J, S, e0, V, T(2.0 * double(mr) / m2), T(2.0 * double(mi) / m2), srcb, e0b, kb);
  // this lane's components of the raw adjoints (contravariant momentum adjoints)
  double* o = G.pbuf + i;
#pragma unroll
  for (int t = 1; t < N; ++t) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int mu = g * C + c;
      o[GradRaw<N>::at(t, mu) * G.count] = double(ls.sg[c] * kb[t - 1][c]);
      o[GradRaw<N>::at(t, 4 + mu) * G.count] = double(srcb[t - 1].re[c]);
      o[GradRaw<N>::at(t, 8 + mu) * G.count] = double(srcb[t - 1].im[c]);
    }
  }
  if (g == 0) o[(GradRaw<N>::words - 1) * G.count] = 1.0;
}

// Second gradient kernel (one lane per event): from the recursion's adjoints that k_grad or
// k_grad_g left in pbuf, the helicity sources' and momenta's adjoints (CM frame), RAMBO's
// conformal map, q(rho) and x1, x2.  Events with |A|^2 = 0 were completed by the first.
template <int N>
__global__ __launch_bounds__(256) void k_grad_back(GradArgs G) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.count) return;
  const double* o = G.pbuf + i;
  if (o[(GradRaw<N>::words - 1) * G.count] == 0.0) return;
  GradKin<N> K;
  grad_front<N>(G, i, K);
  double pb[N][4];
  double rsb = 0.0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) pb[0][mu] = 0.0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = K.leg[t] < 2u ? -K.sc : K.sc;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) pb[t][mu] = sg * o[GradRaw<N>::at(t, mu) * G.count];
    if (K.leg[t] >= 2u) {
      cv4<double> eb;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        eb.re[mu] = o[GradRaw<N>::at(t, 4 + mu) * G.count];
        eb.im[mu] = o[GradRaw<N>::at(t, 8 + mu) * G.count];
      }
      polarisation_adj<double>(K.pc[t], (K.hel >> K.leg[t]) & 1u, eb, pb[t]);
    } else {
      rsb += 0.5 * (pb[t][0] - pb[t][3]);  // leg 1: p = (rs/2)(1, 0, 0, -1)
    }
  }
  grad_back<N>(G, i, K, pb, rsb);
}

}  // namespace bgk
