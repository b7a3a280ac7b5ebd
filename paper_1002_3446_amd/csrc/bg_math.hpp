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

}  // namespace bgk
