// FP64 elementary functions for the event kinematics, callable from host and device code
// (the host build is what the CPU test of their accuracy runs).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace bgk {

// ln 2 as a 42-bit head (so that e * head is exact for every binary exponent e of a double)
// plus the FP64 rounding of the remainder
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;

// Natural logarithm, within about one ulp.  x = m 2^e with m in [sqrt(1/2), sqrt(2));
// f = m - 1 is exact; with s = f / (2 + f), log(1 + f) = 2 atanh(s) = 2 s + s R(s^2) where
// R(z) = sum_{k >= 1} 2 z^k / (2k + 1).  |s| <= 3 - 2 sqrt(2) < 0.1716, so nine terms leave
// a truncation below 3e-17 relative.  Because 2 s = f - s f, log(1 + f) = f - s (f - R):
// the exact f carries the leading part and the rounding of s only touches a term at most
// f / 2 in size.  Then log x = e ln2_hi (exact) + (e ln2_lo + log(1 + f)).  Zero gives
// -inf, negative arguments and NaN give NaN, +inf gives +inf.
__host__ __device__ __forceinline__ double log_fp64(double x) {
  int e = 0;
  double m = std::frexp(x, &e);  // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double R = 2.0 / 19.0;
  R = std::fma(R, z, 2.0 / 17.0);
  R = std::fma(R, z, 2.0 / 15.0);
  R = std::fma(R, z, 2.0 / 13.0);
  R = std::fma(R, z, 2.0 / 11.0);
  R = std::fma(R, z, 2.0 / 9.0);
  R = std::fma(R, z, 2.0 / 7.0);
  R = std::fma(R, z, 2.0 / 5.0);
  R = std::fma(R, z, 2.0 / 3.0);
  R *= z;
  const double lm = f - s * (f - R);
  const double de = (double)e;
  const double r = std::fma(de, kLn2Hi, std::fma(de, kLn2Lo, lm));
  if (x > 0.0 && x < INFINITY) return r;
  return x == 0.0 ? -INFINITY : (x == INFINITY ? x : NAN);
}

// sin(pi t) and cos(pi t) for t in [0, 2] (RAMBO's azimuth, t = 2 rho2), within about two
// ulp and 2^-52 absolute.  k = rint(2 t) picks the quarter period; r = t - k / 2 lies in
// [-1/4, 1/4] and is exact (Sterbenz, or r = t for k = 0).  sin(pi r) and cos(pi r) are
// their Taylor series in z = r^2, whose coefficients (-1)^j pi^(2j+1) / (2j+1)! and
// (-1)^j pi^(2j) / (2j)! are the FP64 roundings of the exact values; with |pi r| <= pi / 4
// the first omitted terms are below 1e-19 (sine, through r^17) and 3e-18 (cosine, through
// r^16).  Then sin(pi t) = sin(pi r + k pi / 2) by the quarter-turn identities.  Arguments
// outside [0, 2] are not reduced further.
__host__ __device__ __forceinline__ void sincospi_fp64(double t, double* sp, double* cp) {
  const double kd = std::rint(2.0 * t);
  const double r = std::fma(kd, -0.5, t);
  const double z = r * r;
  double S = 0x1.aaec32af93359p-21;
  S = std::fma(S, z, -0x1.6fadb9f155744p-16);
  S = std::fma(S, z, 0x1.e8f434d018d63p-12);
  S = std::fma(S, z, -0x1.e3074fde8871fp-8);
  S = std::fma(S, z, 0x1.50783487ee782p-4);
  S = std::fma(S, z, -0x1.32d2cce62bd86p-1);
  S = std::fma(S, z, 0x1.466bc6775aae2p+1);
  S = std::fma(S, z, -0x1.4abbce625be53p+2);
  const double sr = std::fma(r * z, S, r * 0x1.921fb54442d18p+1);
  double C = 0x1.20c62c2f2d7f5p-18;
  C = std::fma(C, z, -0x1.b6e24f44b128fp-14);
  C = std::fma(C, z, 0x1.f9d38a3763cc3p-10);
  C = std::fma(C, z, -0x1.a6d1f2a204a8cp-6);
  C = std::fma(C, z, 0x1.e1f506891babbp-3);
  C = std::fma(C, z, -0x1.55d3c7e3cbffap+0);
  C = std::fma(C, z, 0x1.03c1f081b5ac4p+2);
  C = std::fma(C, z, -0x1.3bd3cc9be45dep+2);
  const double cr = std::fma(z, C, 1.0);
  const int k = (int)kd;
  const double a = (k & 1) ? cr : sr;   // the function that becomes the sine
  const double b = (k & 1) ? sr : cr;
  *sp = (k & 2) ? -a : a;
  *cp = ((k + 1) & 2) ? -b : b;
}

}  // namespace bgk
