// Kernels of the event path: one event per lane, everything for that event kept in the
// lane's registers.  Instantiated per multiplicity N (4..12) and recursion precision T.
#pragma once

#include <type_traits>

#include "bg_device.hpp"
#include "bg_group.hpp"
#include "bg_launch.hpp"
#include "bg_params.hpp"

namespace bgk {

// One event's kinematics: the centre-of-mass momenta in recursion-position order (position 0
// is leg 0, position t >= 1 is leg nib(A, t-1)) for the recursion, and the lab momenta of
// the outgoing gluons in leg order for the cuts and outputs.
template <int N>
struct EventKin {
  double pc[N][4];      // partonic centre-of-mass momenta (RAMBO frame), position order
  double pl[N - 2][4];  // lab momenta of the outgoing legs 2..N-1, leg order
  uint32_t leg[N];      // leg at each position
  uint32_t hel;
  double x1, x2, shat;
};

// Per-lane LDS column through which the outgoing momenta go from leg order to position
// order: slot (4 p + mu) of lane l at perm[(4 p + mu) * stride + l].  Each lane reads only
// what it wrote, so no barrier is needed.
struct PermLds {
  double* col;  // &perm[0][lane]
  int stride;
};

// The column in the kernel's dynamic LDS (launched with perm_lds_bytes(N, blockDim) bytes).
__device__ __forceinline__ PermLds dyn_perm() {
  extern __shared__ double perm_dyn[];
  return PermLds{perm_dyn + threadIdx.x, (int)blockDim.x};
}

// Builds an event's phase-space point (Sec. 3: RAMBO then the longitudinal boost) from
// Philox draws or from caller inputs; writes the optional draw outputs when store is set.
// RAMBO runs over the outgoing legs in leg order (fixed indices, no work for the beams);
// their CM momenta reach the recursion positions through the lane's LDS column.
template <int N>
__device__ __forceinline__ void build_event(const GenClass& C, int64_t i, EventKin<N>& ev, PermLds perm,
                                            bool store = true) {
  constexpr int NF = N - 2;
  const uint64_t e = C.first_event + (uint64_t)i;
  EventRng rng{(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)N, C.key0, C.key1};
  const u32x4 b0 = rng.block(0);

  // colour ordering and helicities
  uint64_t A;
  if (C.in_order) {
    A = 0;
#pragma unroll
    for (int t = 1; t < N; ++t) {
      // a leg index outside 1..N-1 is clamped so that malformed input never addresses
      // outside the event's arrays
      const uint32_t l = C.in_order[i * N + t];
      A |= (uint64_t)(l < 1u ? 1u : (l > (uint32_t)(N - 1) ? (uint32_t)(N - 1) : l)) << (4 * (t - 1));
    }
  } else if (C.random_order) {
    A = shuffle_order<N>(rng);
  } else {
    A = identity_order<N>();
  }
  ev.leg[0] = 0;
#pragma unroll
  for (int t = 1; t < N; ++t) ev.leg[t] = nib(A, t - 1);
  ev.hel = C.in_hel ? C.in_hel[i] : (b0.v[2] & ((1u << N) - 1u));

  // parton fractions
  double sqrt_shat;
  if (C.use_pdf) {
    if (C.in_x) {
      ev.x1 = C.in_x[2 * i];
      ev.x2 = C.in_x[2 * i + 1];
    } else {
      ev.x1 = pdf_sample(u01(b0.v[0]), C.pdf);
      ev.x2 = pdf_sample(u01(b0.v[1]), C.pdf);
    }
    ev.shat = ev.x1 * ev.x2 * C.sqrt_s * C.sqrt_s;
    sqrt_shat = sqrt(ev.shat);
  } else {
    ev.x1 = ev.x2 = 1.0;
    ev.shat = C.sqrt_s * C.sqrt_s;
    sqrt_shat = C.sqrt_s;
  }

  // RAMBO over the outgoing legs: raw q, then the conformal map
  double q[NF][4];
  double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    double r[4];
    if (C.in_u) {
      const double* u = C.in_u + (i * NF + p) * 4;
      r[0] = u[0]; r[1] = u[1]; r[2] = u[2]; r[3] = u[3];
    } else {
      const u32x4 w = rng.block(1u + (uint32_t)p);
      r[0] = u01(w.v[0]); r[1] = u01(w.v[1]); r[2] = u01(w.v[2]); r[3] = u01(w.v[3]);
    }
    rambo_q(r[0], r[1], r[2], r[3], q[p]);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) perm.col[(4 * p + mu) * perm.stride] = q[p][mu];
    if (store && C.out.uniforms) {
      double* uo = C.out.uniforms + (i * NF + p) * 4;
      uo[0] = r[0]; uo[1] = r[1]; uo[2] = r[2]; uo[3] = r[3];
    }
  }
  // Q summed in position order (as the position-order form does, so that every launch form
  // gives bitwise the same momenta)
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const uint32_t j = ev.leg[t];
    const int slot = 4 * (int)(j >= 2u ? j - 2u : 0u);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) Q[mu] += j >= 2u ? perm.col[(slot + mu) * perm.stride] : 0.0;
  }
  RamboMap map;
  map.init(Q, sqrt_shat);
  const double rr = 2.0 * sqrt(ev.x1 * ev.x2);
  const double ch = (ev.x1 + ev.x2) / rr, sh = (ev.x1 - ev.x2) / rr;
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    double pc[4];
    map.apply(q[p], pc);
    ev.pl[p][0] = pc[0] * ch + pc[3] * sh;
    ev.pl[p][1] = pc[1];
    ev.pl[p][2] = pc[2];
    ev.pl[p][3] = pc[3] * ch + pc[0] * sh;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) perm.col[(4 * p + mu) * perm.stride] = pc[mu];
  }
  // positions: beams directly, outgoing legs from the lane's LDS column
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const uint32_t j = ev.leg[t];
    const int slot = 4 * (int)(j >= 2u ? j - 2u : 0u);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) ev.pc[t][mu] = perm.col[(slot + mu) * perm.stride];
    if (j < 2u) {
      ev.pc[t][0] = 0.5 * sqrt_shat; ev.pc[t][1] = 0.0; ev.pc[t][2] = 0.0;
      ev.pc[t][3] = j == 0u ? 0.5 * sqrt_shat : -0.5 * sqrt_shat;
    }
  }
  if (!store) return;
  if (C.out.hel) C.out.hel[i] = ev.hel;
  if (C.out.order) {
#pragma unroll
    for (int t = 0; t < N; ++t) C.out.order[i * N + t] = (uint8_t)ev.leg[t];
  }
  if (C.out.x12) {
    C.out.x12[2 * i] = ev.x1;
    C.out.x12[2 * i + 1] = ev.x2;
  }
  if (C.out.momenta) {
    double* mo = C.out.momenta + i * N * 4;
    const double e1 = 0.5 * C.sqrt_s * ev.x1, e2 = 0.5 * C.sqrt_s * ev.x2;
    mo[0] = e1; mo[1] = 0.0; mo[2] = 0.0; mo[3] = e1;
    mo[4] = e2; mo[5] = 0.0; mo[6] = 0.0; mo[7] = -e2;
#pragma unroll
    for (int p = 0; p < NF; ++p) {
      mo[8 + 4 * p] = ev.pl[p][0]; mo[9 + 4 * p] = ev.pl[p][1];
      mo[10 + 4 * p] = ev.pl[p][2]; mo[11 + 4 * p] = ev.pl[p][3];
    }
  }
}

// eta = asinh(pz / pT) of a massless momentum with energy E and transverse momentum pT, as
// sign(pz) log((E + |pz|) / pT): the same function, since (|p| + |pz|)(|p| - |pz|) = pT^2
// and |p| = E.  E stands in for |p| (the momenta are massless up to rounding, so they agree
// to a few units of 2^-53), which saves the square root.  Every step is a sum of positive
// terms, a division or the logarithm, so the absolute error is a few units of 2^-53 |eta|
// (the cuts and Delta R only use eta through |eta| and differences); pT = 0 gives +-inf.
__device__ __forceinline__ double pseudorapidity(double pt, double pz, double e) {
#pragma clang fp contract(off)
  const double az = fabs(pz);
  return copysign(log_fp64((e + az) / pt), pz);
}

// Jet cuts and observables (Sec. 3, Sec. 4) on the outgoing legs (lab frame).  H_T is summed
// in position order through the lane's LDS column, as the position-order form sums it.
template <int N>
__device__ __forceinline__ bool cuts(const GenClass& C, const EventKin<N>& ev, PermLds perm, double& ht,
                                     double& rmin) {
  // no fused multiply-adds: both forms of the cuts round exactly as written
#pragma clang fp contract(off)
  constexpr int NF = N - 2;
  double pt[NF], eta[NF], phi[NF];
  bool ok = true;
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    const double* m = ev.pl[p];
    pt[p] = sqrt(m[1] * m[1] + m[2] * m[2]);
    eta[p] = pseudorapidity(pt[p], m[3], m[0]);
    phi[p] = atan2(m[2], m[1]);
    perm.col[p * perm.stride] = pt[p];
    ok = ok && (pt[p] > C.pt_min) && (fabs(eta[p]) < C.eta_max);
  }
  ht = 0.0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const uint32_t j = ev.leg[t];
    ht += j >= 2u ? perm.col[(int)(j >= 2u ? j - 2u : 0u) * perm.stride] : 0.0;
  }
  double dr2min = 1e300;
  const double pi = 3.14159265358979323846;
  static_for<0, NF>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    static_for<a + 1, NF>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      double dphi = fabs(phi[a] - phi[b]);
      dphi = dphi > pi ? 2.0 * pi - dphi : dphi;
      const double deta = eta[a] - eta[b];
      dr2min = fmin(dr2min, deta * deta + dphi * dphi);
    });
  });
  rmin = sqrt(dr2min);
  return ok && (dr2min > C.dr_min * C.dr_min);
}

// The same kinematics in recursion-position order throughout (lab momenta of all N legs),
// without the LDS permutation: used where one event spans several lanes, whose register
// budget the leg-order form's extra arrays exceed.
template <int N>
struct EventKinPos {
  double p[N][4];   // physical lab momenta, position order
  double pc[N][4];  // partonic centre-of-mass momenta (RAMBO frame), position order
  uint32_t leg[N];  // leg at each position
  uint32_t hel;
  double x1, x2, shat;
};

// (RAMBO evaluated per position: the beam positions repeat an outgoing leg's draws and are
// overwritten.)
template <int N>
__device__ __forceinline__ void build_event_positions(const GenClass& C, int64_t i, EventKinPos<N>& ev, bool store = true) {
  constexpr int NF = N - 2;
  const uint64_t e = C.first_event + (uint64_t)i;
  EventRng rng{(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)N, C.key0, C.key1};
  const u32x4 b0 = rng.block(0);

  // colour ordering and helicities
  uint64_t A;
  if (C.in_order) {
    A = 0;
#pragma unroll
    for (int t = 1; t < N; ++t) {
      // a leg index outside 1..N-1 is clamped so that malformed input never addresses
      // outside the event's arrays
      const uint32_t l = C.in_order[i * N + t];
      A |= (uint64_t)(l < 1u ? 1u : (l > (uint32_t)(N - 1) ? (uint32_t)(N - 1) : l)) << (4 * (t - 1));
    }
  } else if (C.random_order) {
    A = shuffle_order<N>(rng);
  } else {
    A = identity_order<N>();
  }
  ev.leg[0] = 0;
#pragma unroll
  for (int t = 1; t < N; ++t) ev.leg[t] = nib(A, t - 1);
  ev.hel = C.in_hel ? C.in_hel[i] : (b0.v[2] & ((1u << N) - 1u));

  // parton fractions
  double sqrt_shat;
  if (C.use_pdf) {
    if (C.in_x) {
      ev.x1 = C.in_x[2 * i];
      ev.x2 = C.in_x[2 * i + 1];
    } else {
      ev.x1 = pdf_sample(u01(b0.v[0]), C.pdf);
      ev.x2 = pdf_sample(u01(b0.v[1]), C.pdf);
    }
    ev.shat = ev.x1 * ev.x2 * C.sqrt_s * C.sqrt_s;
    sqrt_shat = sqrt(ev.shat);
  } else {
    ev.x1 = ev.x2 = 1.0;
    ev.shat = C.sqrt_s * C.sqrt_s;
    sqrt_shat = C.sqrt_s;
  }

  // RAMBO in position order: raw q for outgoing legs, then the conformal map
  double q[N][4];
  double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const uint32_t j = ev.leg[t];
    const bool out = j >= 2u;
    const uint32_t pidx = out ? j - 2u : 0u;
    double r[4];
    if (C.in_u) {
      const double* u = C.in_u + (i * NF + pidx) * 4;
      r[0] = u[0]; r[1] = u[1]; r[2] = u[2]; r[3] = u[3];
    } else {
      const u32x4 w = rng.block(1u + pidx);
      r[0] = u01(w.v[0]); r[1] = u01(w.v[1]); r[2] = u01(w.v[2]); r[3] = u01(w.v[3]);
    }
    rambo_q(r[0], r[1], r[2], r[3], q[t]);
    if (out) {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) Q[mu] += q[t][mu];
      if (store && C.out.uniforms) {
        double* uo = C.out.uniforms + (i * NF + pidx) * 4;
        uo[0] = r[0]; uo[1] = r[1]; uo[2] = r[2]; uo[3] = r[3];
      }
    }
  }
  RamboMap map;
  map.init(Q, sqrt_shat);
  const double rr = 2.0 * sqrt(ev.x1 * ev.x2);
  const double ch = (ev.x1 + ev.x2) / rr, sh = (ev.x1 - ev.x2) / rr;
  const double e1 = 0.5 * C.sqrt_s * ev.x1, e2 = 0.5 * C.sqrt_s * ev.x2;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const uint32_t j = ev.leg[t];
    double pc[4];
    map.apply(q[t], pc);  // harmless for beam positions, overwritten below
    double pl[4] = {pc[0] * ch + pc[3] * sh, pc[1], pc[2], pc[3] * ch + pc[0] * sh};
    if (j == 0u) {
      pl[0] = e1; pl[1] = 0.0; pl[2] = 0.0; pl[3] = e1;
      pc[0] = 0.5 * sqrt_shat; pc[1] = 0.0; pc[2] = 0.0; pc[3] = 0.5 * sqrt_shat;
    } else if (j == 1u) {
      pl[0] = e2; pl[1] = 0.0; pl[2] = 0.0; pl[3] = -e2;
      pc[0] = 0.5 * sqrt_shat; pc[1] = 0.0; pc[2] = 0.0; pc[3] = -0.5 * sqrt_shat;
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      ev.p[t][mu] = pl[mu];
      ev.pc[t][mu] = pc[mu];
    }
  }
  if (!store) return;
  if (C.out.hel) C.out.hel[i] = ev.hel;
  if (C.out.order) {
#pragma unroll
    for (int t = 0; t < N; ++t) C.out.order[i * N + t] = (uint8_t)ev.leg[t];
  }
  if (C.out.x12) {
    C.out.x12[2 * i] = ev.x1;
    C.out.x12[2 * i + 1] = ev.x2;
  }
  if (C.out.momenta) {
#pragma unroll
    for (int t = 0; t < N; ++t) {
      double* mo = C.out.momenta + (i * N + ev.leg[t]) * 4;
      mo[0] = ev.p[t][0]; mo[1] = ev.p[t][1]; mo[2] = ev.p[t][2]; mo[3] = ev.p[t][3];
    }
  }
}

// cuts() on position-ordered lab momenta (the beam positions masked).
template <int N>
__device__ __forceinline__ bool cuts_positions(const GenClass& C, const EventKinPos<N>& ev, double& ht, double& rmin) {
#pragma clang fp contract(off)
  double pt[N], eta[N], phi[N];
  bool ok = true;
  ht = 0.0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double* p = ev.p[t];
    pt[t] = sqrt(p[1] * p[1] + p[2] * p[2]);
    eta[t] = pseudorapidity(pt[t], p[3], p[0]);
    phi[t] = atan2(p[2], p[1]);
    const bool out = ev.leg[t] >= 2u;
    if (out) {
      ht += pt[t];
      ok = ok && (pt[t] > C.pt_min) && (fabs(eta[t]) < C.eta_max);
    }
  }
  double dr2min = 1e300;
  const double pi = 3.14159265358979323846;
  static_for<1, N>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    static_for<t + 1, N>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      double dphi = fabs(phi[t] - phi[u]);
      dphi = dphi > pi ? 2.0 * pi - dphi : dphi;
      const double deta = eta[t] - eta[u];
      const double d2 = deta * deta + dphi * dphi;
      const bool both = (ev.leg[t] >= 2u) && (ev.leg[u] >= 2u);
      dr2min = both ? fmin(dr2min, d2) : dr2min;
    });
  });
  rmin = sqrt(dr2min);
  return ok && (dr2min > C.dr_min * C.dr_min);
}

// |A(sigma;h)|^2 from position-ordered physical momenta.  Momenta are scaled by the power
// of two 2^-ex nearest below half their summed energy (exact in binary floating point),
// and |A|^2(k) = 2^(2 ex (4-N)) |A|^2(2^-ex k).
template <int N, typename T>
struct UseLdsK {
  static constexpr bool value = lds_span_table(N, std::is_same<T, float>::value ? 32 : 64);
};

// The LDS span table of one workgroup (only instantiated where UseLdsK holds).
template <int N>
struct LdsTable {
  float4 k[Spans<N - 1>::count * kLdsLanes];
  float p[Spans<N - 1>::count * kLdsLanes];
};

template <int N, typename T, bool LDS>
__device__ __forceinline__ double ordered_amp2(const double (&p)[N][4], const uint32_t (&leg)[N], uint32_t hel,
                                               LdsTable<N>* tab) {
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) esum += fabs(p[t][0]);
  const int ex = ilogb(0.5 * esum);
  const double sc = ldexp(1.0, -ex);
  double k[N - 1][4];
  cv4<T> src[N - 1];
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = leg[t] < 2u ? -sc : sc;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) k[t - 1][mu] = sg * p[t][mu];
    src[t - 1] = polarisation<T>(p[t], (hel >> leg[t]) & 1u);
  }
  const cv4<T> e0 = polarisation<T>(p[0], (hel >> leg[0]) & 1u);
  double mr, mi;
  if constexpr (LDS) {
    // the generation kernel carries its momentum permutation (doubles) in this memory: the
    // barrier keeps the compiler from moving the table fill above those accesses (the
    // workgroup is one wave, so it costs nothing else)
    __syncthreads();
    SpanKLds<N - 1, kLdsLanes> ks{tab->k + threadIdx.x, tab->p + threadIdx.x};
    ks.fill(k);
    bg_amplitude<N - 1, T>(ks, src, e0, mr, mi);
  } else {
    SpanKLegs<N - 1, T> ks{k};
    bg_amplitude<N - 1, T>(ks, src, e0, mr, mi);
  }
  return ldexp(__builtin_fma(mr, mr, mi * mi), 2 * ex * (4 - N) - (N - 2));
}

// Angles of the real polarisations of an event (random_polarisation): leg k takes word k % 4
// of Philox block n_blocks + k / 4 (after the draws of the helicity mode), psi = 2 pi u;
// returns cos psi, sin psi per leg, evaluated in FP64.
template <int N>
__device__ __forceinline__ void polarisation_angles(const GenClass& C, int64_t i, double (&cs)[N][2]) {
  const uint64_t e = C.first_event + (uint64_t)i;
  const EventRng rng{(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)N, C.key0, C.key1};
  constexpr uint32_t b0 = 1u + (N - 2) + (N - 2 + 3) / 4;
  u32x4 w{};
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if ((k & 3) == 0) w = rng.block(b0 + (uint32_t)(k / 4));
    sincospi_fp64(2.0 * u01(w.v[k & 3]), &cs[k][1], &cs[k][0]);
  }
}

// |A(sigma; eps_psi)|^2 with real polarisations (cs: cos, sin of each leg's angle), as
// ordered_amp2.
template <int N, typename T, bool LDS>
__device__ __forceinline__ double ordered_amp2_real(const double (&p)[N][4], const uint32_t (&leg)[N],
                                                    const double (&cs)[N][2], LdsTable<N>* tab) {
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) esum += fabs(p[t][0]);
  const int ex = ilogb(0.5 * esum);
  const double sc = ldexp(1.0, -ex);
  double k[N - 1][4];
  rv4<T> src[N - 1];
  // the angle of the leg at each position, selected without dynamic register indexing
  auto angle = [&](uint32_t l, T& c, T& s) {
    double cd = cs[0][0], sd = cs[0][1];
#pragma unroll
    for (int q = 1; q < N; ++q) {
      cd = l == (uint32_t)q ? cs[q][0] : cd;
      sd = l == (uint32_t)q ? cs[q][1] : sd;
    }
    c = T(cd);
    s = T(sd);
  };
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = leg[t] < 2u ? -sc : sc;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) k[t - 1][mu] = sg * p[t][mu];
    T c, s;
    angle(leg[t], c, s);
    src[t - 1] = real_polarisation<T>(p[t], c, s);
  }
  T c0, s0;
  angle(leg[0], c0, s0);
  const rv4<T> e0 = real_polarisation<T>(p[0], c0, s0);
  double m;
  if constexpr (LDS) {
    __syncthreads();
    SpanKLds<N - 1, kLdsLanes> ks{tab->k + threadIdx.x, tab->p + threadIdx.x};
    ks.fill(k);
    m = bg_amplitude_r<N - 1, T>(ks, src, e0);
  } else {
    SpanKLegs<N - 1, T> ks{k};
    m = bg_amplitude_r<N - 1, T>(ks, src, e0);
  }
  return ldexp(m * m, 2 * ex * (4 - N) - (N - 2));
}

// The same with the event spread over the G lanes of a group; g is this lane's place in it.
// With ktab (this lane's column of a workgroup table of span_k_lds_bytes per lane, row
// stride `lanes`), the span momenta come from LDS (SpanKGroupLds), else from registers.
// Whether the grouped forward recursion forms each span momentum afresh at every use (FP64
// with two lanes from n = 9, with four from n = 11): keeping every span's sums live would
// spill there (n = 12, four lanes: 656 against 400 B of scratch per lane; n = 9, two lanes:
// 512 against 288 B), and the extra FP64 additions cost less than the spill traffic.
template <int N, typename T, int G>
constexpr bool fwd_afresh() { return std::is_same<T, double>::value && (N >= 11 || (G == 2 && N >= 9)); }

template <int N, typename T, int G, bool KLDS = false>
__device__ __forceinline__ double ordered_amp2_g(const double (&p)[N][4], const uint32_t (&leg)[N], uint32_t hel,
                                                 int g, T* ktab = nullptr, int lanes = 0) {
  constexpr int C = 4 / G;
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) esum += fabs(p[t][0]);
  const int ex = ilogb(0.5 * esum);
  const double sc = ldexp(1.0, -ex);
  const LaneShare<G, T> ls(g);
  const LaneShare<G, double> lsd(g);
  double k[N - 1][C];  // covariant, this lane's components
  cvl<T, C> src[N - 1], e0;
#pragma unroll
  for (int t = 1; t < N; ++t) {
    const double sg = leg[t] < 2u ? -sc : sc;
#pragma unroll
    for (int c = 0; c < C; ++c) k[t - 1][c] = lsd.sg[c] * (sg * lsd.pick(p[t], c));
    const cv4<T> e = polarisation<T>(p[t], (hel >> leg[t]) & 1u);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      src[t - 1].re[c] = ls.pick(e.re, c);
      src[t - 1].im[c] = ls.pick(e.im, c);
    }
  }
  {
    const cv4<T> e = polarisation<T>(p[0], (hel >> leg[0]) & 1u);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      e0.re[c] = ls.pick(e.re, c);
      e0.im[c] = ls.pick(e.im, c);
    }
  }
  double mr, mi;
  if constexpr (KLDS) {
    const SpanKGroupLds<N - 1, G, T> ks(k, lsd.sg, ktab, lanes);
    ks.fill();
    bg_amplitude_g<N - 1, G, T>(ls, ks, src, e0, mr, mi);
  } else {
    const SpanKGroup<N - 1, G, T, fwd_afresh<N, T, G>()> ks{k, lsd.sg};
    bg_amplitude_g<N - 1, G, T>(ls, ks, src, e0, mr, mi);
  }
  return ldexp(__builtin_fma(mr, mr, mi * mi), 2 * ex * (4 - N) - (N - 2));
}

// Compensated (sum w, sum w^2) of a workgroup of up to 256 lanes, in a fixed tree order;
// thread 0 stores (s, c, s2, c2) to dst.
__device__ __forceinline__ void block_reduce_store(CSum w, CSum w2, double* dst) {
  __shared__ double red[4][4];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    CSum ow{__shfl_down(w.s, off), __shfl_down(w.c, off)};
    CSum ow2{__shfl_down(w2.s, off), __shfl_down(w2.c, off)};
    w = cs_add(w, ow);
    w2 = cs_add(w2, ow2);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = w.s; red[wave][1] = w.c; red[wave][2] = w2.s; red[wave][3] = w2.c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    CSum a{red[0][0], red[0][1]}, b{red[0][2], red[0][3]};
    const int nw = (int)(blockDim.x >> 6);
    for (int v = 1; v < nw; ++v) {
      a = cs_add(a, CSum{red[v][0], red[v][1]});
      b = cs_add(b, CSum{red[v][2], red[v][3]});
    }
    dst[0] = a.s; dst[1] = a.c; dst[2] = b.s; dst[3] = b.c;
  }
}

// The weight of Eq. 3.8 from |A|^2 (w = 0 exactly when the event fails the cuts, never
// 0 times a product), and the per-event outputs of |A|^2, the weight, the cut flag and the
// log integrand weight; returns w.  Shared by every generation kernel, so that each
// output rounds identically whichever kernel evaluates the event.
// Dynamic scale mu = H_T: alpha_s(mu)^(n-2) f(x1, mu) f(x2, mu) over the factors at mu0 that
// wconst and the sampling density hold (exactly 1 with a fixed scale).
template <int N>
__device__ __forceinline__ double scale_ratio(const GenClass& C, double ht, double x1, double x2) {
#pragma clang fp contract(off)
  if (!C.dynamic_scale) return 1.0;
  const double lmu = log(ht);
  double lr = double(N - 2) * (log(grid_alpha(C.grid, lmu)) - C.log_alpha0);
  if (C.use_pdf) {
    const double l1 = log(x1), l2 = log(x2), m1 = log1p(-x1), m2 = log1p(-x2);
    lr += (grid_lnf(C.grid, lmu, l1 - m1) - (C.pdf.a * l1 + double(C.pdf.b) * m1)) +
          (grid_lnf(C.grid, lmu, l2 - m2) - (C.pdf.a * l2 + double(C.pdf.b) * m2));
  }
  return exp(lr);
}

// r: scale_ratio of the event.
template <int N>
__device__ __forceinline__ double finish_event(const GenClass& C, int64_t i, bool pass, double a2, double shat,
                                               double x1, double x2, double r) {
#pragma clang fp contract(off)
  double sp = 1.0;
#pragma unroll
  for (int k = 0; k < (N > 5 ? N - 5 : 5 - N); ++k) sp *= shat;
  if (N < 5) sp = 1.0 / sp;
  const double w = pass ? C.wconst * sp * a2 * r : 0.0;
  if (C.out.weight) C.out.weight[i] = w;
  if (C.out.amp2) C.out.amp2[i] = a2;
  if (C.out.pass) C.out.pass[i] = pass ? 1 : 0;
  if (C.out.logw) {
    double lw = log(a2) + double(N - 5) * log(shat) + C.log_const;
    if (C.use_pdf) lw += C.pdf.a * (log(x1) + log(x2)) + double(C.pdf.b) * (log1p(-x1) + log1p(-x2));
    if (C.dynamic_scale) lw += log(r);
    C.out.logw[i] = a2 > 0.0 ? lw : -INFINITY;
  }
  return w;
}

// One event: draws -> kinematics -> cuts -> |A|^2 -> weight; writes outputs; returns w.
// With G > 1 lanes per event every lane of the group evaluates the kinematics (the same
// values), the recursion is shared, and lane g = 0 writes the outputs and returns w
// (the others return 0).  Not used for the table classes, which run split (bg_split.hpp).
template <int N, typename T, int G = 1, int POL = 0, bool KLDS = false>
__device__ __forceinline__ double generate_one(const GenClass& C, int64_t i, PermLds perm, int g = 0,
                                               T* ktab = nullptr, int lanes = 0) {
  static_assert(POL == 0 || G == 1, "real polarisations run one lane per event");
  using Kin = typename std::conditional<G == 1, EventKin<N>, EventKinPos<N>>::type;
  Kin ev;
  double ht, rmin;
  bool pass;
  if constexpr (G == 1) {
    build_event<N>(C, i, ev, perm, g == 0);
    pass = cuts<N>(C, ev, perm, ht, rmin);
  } else {
    (void)perm;
    build_event_positions<N>(C, i, ev, g == 0);
    pass = cuts_positions<N>(C, ev, ht, rmin);
  }
  // |A|^2 is Lorentz invariant: evaluated in the partonic centre-of-mass frame
  double a2;
  if constexpr (POL == 1) {
    double cs[N][2];
    polarisation_angles<N>(C, i, cs);
    a2 = ordered_amp2_real<N, T, false>(ev.pc, ev.leg, cs, nullptr);
  } else if constexpr (G == 1) {
    a2 = ordered_amp2<N, T, false>(ev.pc, ev.leg, ev.hel, nullptr);
  } else {
    a2 = ordered_amp2_g<N, T, G, KLDS>(ev.pc, ev.leg, ev.hel, g, ktab, lanes);
  }
  if (g != 0) return 0.0;
  if (C.out.obs) {
    C.out.obs[2 * i] = ht;
    C.out.obs[2 * i + 1] = rmin;
  }
  return finish_event<N>(C, i, pass, a2, ev.shat, ev.x1, ev.x2, scale_ratio<N>(C, ht, ev.x1, ev.x2));
}

// Single-class generation of a class without the span table (FP32 n = 9, FP64 n <= 6): one
// event per lane, one compensated partial per workgroup.  Launch: blockDim.x in
// {64, 128, 192, 256} with perm_lds_bytes(N, blockDim.x) bytes of dynamic LDS; partials may
// be NULL.
template <int N, typename T, int POL = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_generate(GenClass C,
                                                                                            double* partials) {
  static_assert(!UseLdsK<N, T>::value, "the table classes generate in the split form");
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  if (i < C.count) w = generate_one<N, T, 1, POL>(C, i, dyn_perm());
  if (partials) block_reduce_store(CSum{w, 0.0}, CSum{w * w, 0.0}, partials + 4 * (int64_t)blockIdx.x);
}

// |A|^2 from given momenta (bg_amp2): momenta [count][N][4] physical, gathered in colour order.
template <int N, typename T>
__global__ __launch_bounds__((UseLdsK<N, T>::value ? kLdsLanes : 256)) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_amp2(int64_t count, const double* __restrict__ mom,
                                                const uint32_t* __restrict__ hel,
                                                const uint8_t* __restrict__ order,
                                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double p[N][4];
  uint32_t leg[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const uint32_t l = order[i * N + t];
    leg[t] = l < (uint32_t)N ? l : (uint32_t)(N - 1);  // malformed input stays in bounds
    const double* q = mom + (i * N + leg[t]) * 4;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) p[t][mu] = q[mu];
  }
  if constexpr (UseLdsK<N, T>::value) {
    __shared__ LdsTable<N> tab;
    out[i] = ordered_amp2<N, T, true>(p, leg, hel[i], &tab);
  } else {
    out[i] = ordered_amp2<N, T, false>(p, leg, hel[i], nullptr);
  }
}

// Whether the grouped recursion of precision T reads its span momenta from the LDS table:
// in FP32 it replaces FP64 sums and conversions at every use; in FP64, whose currents fill
// the registers, the table's reads add to the scratch spill, so FP64 sums in registers.
template <typename T>
constexpr bool span_k_table() {
  return sizeof(T) == 4;
}

// Dynamic LDS of the grouped kernels for workgroups of `block` lanes: the span-momentum table
template <int N, typename T, int G>
constexpr int grouped_lds_bytes(int block) {
  return span_k_table<T>() ? span_k_lds_bytes<N - 1, G, T>() * block : 0;
}

// bg_amp2 with G lanes per event.  Dynamic LDS: grouped_lds_bytes.
template <int N, typename T, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_amp2_g(
    int64_t count, const double* __restrict__ mom, const uint32_t* __restrict__ hel, const uint8_t* __restrict__ order,
    double* __restrict__ out) {
  extern __shared__ unsigned char gdyn[];
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int g = (int)(threadIdx.x % G);
  if (i >= count) return;
  double p[N][4];
  uint32_t leg[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const uint32_t l = order[i * N + t];
    leg[t] = l < (uint32_t)N ? l : (uint32_t)(N - 1);  // malformed input stays in bounds
    const double* q = mom + (i * N + leg[t]) * 4;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) p[t][mu] = q[mu];
  }
  const double a2 = ordered_amp2_g<N, T, G, span_k_table<T>()>(p, leg, hel[i], g,
                                                               reinterpret_cast<T*>(gdyn) + threadIdx.x,
                                                               (int)blockDim.x);
  if (g == 0) out[i] = a2;
}

}  // namespace bgk
