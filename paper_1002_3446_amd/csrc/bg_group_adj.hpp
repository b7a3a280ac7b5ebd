// Reverse sweep of the grouped recursion (bg_group.hpp): the adjoint of the forward pass with
// one event spread over G lanes, each lane holding C = 4 / G Lorentz components of every
// current and of every current's adjoint.  Scalar adjoints that come from a sum over all
// components (conj(J).Jbar-type contractions) are completed across the group with the
// same DPP sums as the forward products, so every lane of a group holds identical scalar
// adjoints; vector adjoints stay per lane.  Complex adjoints follow the convention of the
// one-lane adjoint: zbar = dL/dRe z + i dL/dIm z, and w = x y gives xbar += conj(y) wbar.
#pragma once

#include "bg_group.hpp"

namespace bgk {

// cb += sum over all components of conj(y) . accb (group-complete)
template <int G, typename T, int C>
__device__ __forceinline__ void conj_dot_g(const cvl<T, C>& y, const cvl<T, C>& accb, T& cbr, T& cbi) {
  T r = y.re[0] * accb.re[0], i = y.re[0] * accb.im[0];
  r = fmac(y.im[0], accb.im[0], r);
  i = fmac(-y.im[0], accb.re[0], i);
#pragma unroll
  for (int c = 1; c < C; ++c) {
    r = fmac(y.re[c], accb.re[c], fmac(y.im[c], accb.im[c], r));
    i = fmac(y.re[c], accb.im[c], fmac(-y.im[c], accb.re[c], i));
  }
  cbr += group_sum<G>(r);
  cbi += group_sum<G>(i);
}

// yb += conj(c) accb  (from acc += c y)
template <typename T, int C>
__device__ __forceinline__ void axpy_adj_y(T cr, T ci, const cvl<T, C>& accb, cvl<T, C>& yb) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    yb.re[c] = fmac(ci, accb.im[c], fmac(cr, accb.re[c], yb.re[c]));
    yb.im[c] = fmac(-ci, accb.re[c], fmac(cr, accb.im[c], yb.im[c]));
  }
}

// xb_c += sigma_c conj(y_c) db  (from d = x . y with the metric)
template <int G, typename T, int C>
__device__ __forceinline__ void mdot_adj(const LaneShare<G, T>& ls, const cvl<T, C>& y, T dbr, T dbi, cvl<T, C>& xb) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const T yr = ls.sg[c] * y.re[c], yi = ls.sg[c] * y.im[c];
    xb.re[c] = fmac(yi, dbi, fmac(yr, dbr, xb.re[c]));
    xb.im[c] = fmac(-yi, dbr, fmac(yr, dbi, xb.im[c]));
  }
}

// add a covariant span-momentum adjoint (this lane's components) to each of the legs A..B
template <int A, int B, int L, typename T, int C>
__device__ __forceinline__ void spread_g(const T (&Kb)[C], T (&kb)[L][C]) {
  static_for<A, B + 1>([&](auto tc) {
#pragma unroll
    for (int c = 0; c < C; ++c) kb[decltype(tc)::value][c] += Kb[c];
  });
}

// Reverse of span_vertex_g for span [A..B]: given Vb (adjoint of the bracket sum, this lane's
// components) and the adjoint (sbr, sbi) of its span scalar, accumulate into the adjoints of
// the sub-currents, sub-span scalars and covariant leg momenta.
template <int L, int A, int B, int G, typename T, typename KS, typename SS>
__device__ __forceinline__ void span_vertex_adj_g(const LaneShare<G, T>& ls, const KS& ks,
                                                  const cvl<T, 4 / G> (&J)[Spans<L>::count], const SS& S,
                                                  const cvl<T, 4 / G>& Vb, T sbr, T sbi,
                                                  cvl<T, 4 / G> (&Jb)[Spans<L>::count], SS& Sb, T (&kb)[L][4 / G]) {
  constexpr int C = 4 / G;
  using SP = Spans<L>;
  // V = 2X + sigma Yc + Z
  cvl<T, C> Xb, Ycb;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    Xb.re[c] = T(2) * Vb.re[c];
    Xb.im[c] = T(2) * Vb.im[c];
    Ycb.re[c] = ls.sg[c] * Vb.re[c];
    Ycb.im[c] = ls.sg[c] * Vb.im[c];
  }
  const cvl<T, C>& Zb = Vb;
  // Z -= S[A..j] J[j+1..B]  and  Z -= S[i+1..B] J[A..i]
  static_for<A + 1, B>([&](auto jc) {
    constexpr int j = decltype(jc)::value, Sx = SP::at(A, j), Jx = SP::at(j + 1, B);
    T cr = T(0), ci = T(0);
    conj_dot_g<G>(J[Jx], Zb, cr, ci);
    Sb.template sub<Sx>(cr, ci);
    T sr, si;
    S.template get<Sx>(sr, si);
    axpy_adj_y(-sr, -si, Zb, Jb[Jx]);
  });
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value, Sx = SP::at(i + 1, B), Jx = SP::at(A, i);
    T cr = T(0), ci = T(0);
    conj_dot_g<G>(J[Jx], Zb, cr, ci);
    Sb.template sub<Sx>(cr, ci);
    T sr, si;
    S.template get<Sx>(sr, si);
    axpy_adj_y(-sr, -si, Zb, Jb[Jx]);
  });
  // X += (J[A..i] . J[j+1..B]) J[i+1..j]
  static_for<A, B - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    static_for<i + 1, B>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int PA = SP::at(A, i), PM = SP::at(i + 1, j), PC = SP::at(j + 1, B);
      T er, ei;
      cdot_g<G>(ls, J[PA], J[PC], er, ei);
      T ebr = T(0), ebi = T(0);
      conj_dot_g<G>(J[PM], Xb, ebr, ebi);
      axpy_adj_y(er, ei, Xb, Jb[PM]);
      mdot_adj(ls, J[PC], ebr, ebi, Jb[PA]);
      mdot_adj(ls, J[PA], ebr, ebi, Jb[PC]);
    });
  });
  // three-gluon brackets
  static_for<A, B>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int PA = SP::at(A, i), PB = SP::at(i + 1, B);
    T ka[C], kbv[C];
    ks.template K<A, i>(ka);
    ks.template K<i + 1, B>(kbv);
    T dr, di, ar, ai, br, bi;
    cdot_g<G>(ls, J[PA], J[PB], dr, di);
    rdot_g<G>(J[PA], kbv, ar, ai);
    rdot_g<G>(J[PB], ka, br, bi);
    // X += a J[PB] - b J[PA]
    T abr = T(0), abi = T(0), bbr = T(0), bbi = T(0);
    conj_dot_g<G>(J[PB], Xb, abr, abi);
    axpy_adj_y(ar, ai, Xb, Jb[PB]);
    conj_dot_g<G>(J[PA], Xb, bbr, bbi);
    bbr = -bbr;
    bbi = -bbi;
    axpy_adj_y(-br, -bi, Xb, Jb[PA]);
    // Yc += d (KA - KB);  S += d
    T dbr = T(0), dbi = T(0);
    T KAb[C], KBb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const T dk = ka[c] - kbv[c];
      dbr = fmac(dk, Ycb.re[c], dbr);
      dbi = fmac(dk, Ycb.im[c], dbi);
      const T w = fmac(dr, Ycb.re[c], di * Ycb.im[c]);  // Re(conj(d) Ycb_c)
      KAb[c] = w;
      KBb[c] = -w;
    }
    dbr = sbr + group_sum<G>(dbr);
    dbi = sbi + group_sum<G>(dbi);
    // d = J[PA] . J[PB]
    mdot_adj(ls, J[PB], dbr, dbi, Jb[PA]);
    mdot_adj(ls, J[PA], dbr, dbi, Jb[PB]);
    // a = J[PA] . KB,  b = J[PB] . KA  (covariant K: no metric signs)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      Jb[PA].re[c] = fmac(kbv[c], abr, Jb[PA].re[c]);
      Jb[PA].im[c] = fmac(kbv[c], abi, Jb[PA].im[c]);
      KBb[c] = fmac(J[PA].re[c], abr, fmac(J[PA].im[c], abi, KBb[c]));
      Jb[PB].re[c] = fmac(ka[c], bbr, Jb[PB].re[c]);
      Jb[PB].im[c] = fmac(ka[c], bbi, Jb[PB].im[c]);
      KAb[c] = fmac(J[PB].re[c], bbr, fmac(J[PB].im[c], bbi, KAb[c]));
    }
    spread_g<A, i, L>(KAb, kb);
    spread_g<i + 1, B, L>(KBb, kb);
  });
}

// Reverse sweep of bg_forward_g + closure.  mb: adjoint of m = eps0 . V (identical on the
// lanes of a group).  Outputs the adjoints of the sources (srcb), of the closing polarisation
// (e0b) and of the scaled covariant leg momenta (kb), this lane's components.
template <int L, int G, typename T, typename KS, typename SS>
__device__ __forceinline__ void bg_reverse_g(const LaneShare<G, T>& ls, const KS& ks,
                                             const cvl<T, 4 / G> (&J)[Spans<L>::count], const SS& S,
                                             const cvl<T, 4 / G>& eps0, const cvl<T, 4 / G>& Vfull, T mbr, T mbi,
                                             cvl<T, 4 / G> (&srcb)[L], cvl<T, 4 / G>& e0b, T (&kb)[L][4 / G]) {
  constexpr int C = 4 / G;
  using SP = Spans<L>;
  cvl<T, C> Jb[SP::count];
  SS Sb(S.g);
  Sb.zero();
  static_for<0, SP::count>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
#pragma unroll
    for (int c = 0; c < C; ++c) Jb[s].re[c] = Jb[s].im[c] = T(0);
  });
  static_for<0, L>([&](auto tc) {
#pragma unroll
    for (int c = 0; c < C; ++c) kb[decltype(tc)::value][c] = T(0);
  });
  cvl<T, C> Vb;
#pragma unroll
  for (int c = 0; c < C; ++c) Vb.re[c] = Vb.im[c] = e0b.re[c] = e0b.im[c] = T(0);
  mdot_adj(ls, eps0, mbr, mbi, Vb);
  mdot_adj(ls, Vfull, mbr, mbi, e0b);
  span_vertex_adj_g<L, 0, L - 1, G, T>(ls, ks, J, S, Vb, T(0), T(0), Jb, Sb, kb);
  // lengths L-1 down to 2
  static_for<0, L - 2>([&](auto rc) {
    constexpr int len = L - 1 - decltype(rc)::value;
    static_for<0, L - len + 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value, b = a + len - 1, s = SP::at(a, b);
      T Kc[C];
      ks.template K<a, b>(Kc);
      const T prop = ks.template prop<a, b>();
      // J = V prop:  Vb = prop Jb;  K_mu (covariant) gets -2 sigma_mu K_mu prop sum Re(conj(J) Jb)
      cvl<T, C> Vbs;
      T rj = T(0);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        Vbs.re[c] = prop * Jb[s].re[c];
        Vbs.im[c] = prop * Jb[s].im[c];
        rj = fmac(J[s].re[c], Jb[s].re[c], fmac(J[s].im[c], Jb[s].im[c], rj));
      }
      rj = group_sum<G>(rj);
      T Kb[C];
#pragma unroll
      for (int c = 0; c < C; ++c) Kb[c] = T(-2) * ls.sg[c] * Kc[c] * prop * rj;
      spread_g<a, b, L>(Kb, kb);
      T sbr, sbi;
      Sb.template get<s>(sbr, sbi);
      span_vertex_adj_g<L, a, b, G, T>(ls, ks, J, S, Vbs, sbr, sbi, Jb, Sb, kb);
    });
  });
  static_for<0, L>([&](auto tc) { srcb[decltype(tc)::value] = Jb[decltype(tc)::value]; });
}

// The full four-vector from the lanes' shares (G = 2): own components and the partner's.
template <typename U>
__device__ __forceinline__ void gather_pair(int g, const U (&own)[2], U (&full)[4]) {
  U other[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) other[c] = dpp_mov<kDppSwap1>(own[c]);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    full[c] = g == 0 ? own[c] : other[c];
    full[2 + c] = g == 0 ? other[c] : own[c];
  }
}

}  // namespace bgk
