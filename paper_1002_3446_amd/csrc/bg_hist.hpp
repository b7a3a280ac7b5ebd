// Exact per-bin sums of event weights, for the distributions of Sec. 4 (Fig. 3: H_T and
// R_min) and the convergence study of Fig. 2, on the device.
//
// The paper histograms on the CPU and sums with Kahan's algorithm to avoid the drift of a
// naive sum over ~1e11 weights (Sec. 4).  Here every bin accumulates its sum w and sum w^2
// EXACTLY, in fixed point: a non-negative double x = m 2^e (m a 53-bit integer) is an integer
// multiple of 2^kHistFloor, and its bits, cut at 32-bit boundaries of that grid, are added to
// kHistLimbs signed 64-bit limbs (limb j counts units of 2^(kHistFloor + 32 j)).  Integer
// addition is exact and associative, so atomic adds in any order give the same limbs: the
// totals are deterministic and, read out with one correct rounding (hist_limbs_to_double),
// equal the correctly rounded exact sums (what math.fsum returns).  Bits below 2^kHistFloor
// (2^-160, far below any weight in pb) are dropped; values of 2^224 or more are rejected.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgk {

constexpr int kHistLimbs = 12;    // 384 bits
constexpr int kHistFloor = -160;  // exponent of limb 0's unit

// Adds the exact bits of x >= 0 (finite) to limbs[0..kHistLimbs-1] through add(j, chunk),
// each chunk in [0, 2^32); returns false (adding nothing) for a value of 2^224 or more or a
// non-finite or negative one.
template <typename Add>
__host__ __device__ inline bool hist_split(double x, Add&& add) {
  if (!(x >= 0.0) || !(x < 0x1p224)) return false;
  if (x == 0.0) return true;
  int E;
  const double f = frexp(x, &E);            // x = f 2^E, f in [1/2, 1)
  uint64_t m = (uint64_t)ldexp(f, 53);      // exact: 53-bit integer
  int p0 = E - 53 - kHistFloor;             // grid position of m's lowest bit
  if (p0 < 0) {
    if (p0 <= -53) return true;             // below the grid entirely
    m >>= -p0;                              // drop the bits below 2^kHistFloor
    p0 = 0;
  }
  const int j0 = p0 >> 5, q = p0 & 31;
  const uint64_t lo = m << q;               // bits 0..63 of m 2^q
  const uint64_t hi = q > 11 ? m >> (64 - q) : 0;  // bits 64..84
  if ((lo & 0xFFFFFFFFull) != 0) add(j0, (int64_t)(lo & 0xFFFFFFFFull));
  if ((lo >> 32) != 0) add(j0 + 1, (int64_t)(lo >> 32));
  if (hi != 0) add(j0 + 2, (int64_t)hi);
  return true;
}

// Carry-propagates limbs in place: limbs 0..kHistLimbs-2 into [0, 2^32), the rest into the
// top limb.  The limbs hold a non-negative total, so the top limb ends non-negative.
__host__ __device__ inline void hist_normalise(int64_t* L) {
  for (int j = 0; j < kHistLimbs - 1; ++j) {
    const int64_t c = L[j] >> 32;           // floor division by 2^32 (arithmetic shift)
    L[j] -= c * (int64_t(1) << 32);
    L[j + 1] += c;
  }
}

// The correctly rounded (to nearest, ties to even) double of normalised limbs.
__host__ __device__ inline double hist_limbs_to_double(const int64_t* L) {
  int t = kHistLimbs - 1;
  while (t >= 0 && L[t] == 0) --t;
  if (t < 0) return 0.0;
  // the top 96 bits as (a: limb t, b: limbs t-1, t-2), the rest as a sticky flag
  const uint64_t a = (uint64_t)L[t];
  const uint64_t b1 = t >= 1 ? (uint64_t)L[t - 1] : 0, b2 = t >= 2 ? (uint64_t)L[t - 2] : 0;
  bool sticky = false;
  for (int j = t - 3; j >= 0; --j) sticky = sticky || L[j] != 0;
  // v = a 2^64 + b1 2^32 + b2 (a may exceed 32 bits only in the top limb)
  int lz = 0;
  while (lz < 64 && !((a >> (63 - lz)) & 1u)) ++lz;
  // top 64 bits of v, left-aligned, and the bits below them
  const uint64_t b = (b1 << 32) | b2;
  uint64_t top;
  uint64_t rest;
  if (lz == 0) {
    top = a;
    rest = b;
  } else {
    top = (a << lz) | (b >> (64 - lz));
    rest = b << lz;
  }
  sticky = sticky || rest != 0;
  // round top (64 bits, leading bit set) to 53 bits
  uint64_t mant = top >> 11;
  const uint64_t rbits = top & 0x7FFull;    // the 11 discarded bits
  const bool half = (rbits >> 10) & 1u;
  const bool below = (rbits & 0x3FFull) != 0 || sticky;
  if (half && (below || (mant & 1u))) ++mant;
  // value = mant 2^(exponent of top's lowest kept bit)
  const int e = kHistFloor + 32 * (t - 2) + 64 - lz + 11;  // position of mant's unit
  return ldexp((double)mant, e);
}

}  // namespace bgk
