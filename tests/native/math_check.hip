// Host-side driver for the accuracy test of the library's FP64 elementary functions:
// prints, in hexadecimal, "L x log(x)" for arguments spread over many binades and
// "S t sin(pi t) cos(pi t)" for t over [0, 2] (uniform, near the quarter-period seams, and
// the seams themselves).
#include <cstdint>
#include <cstdio>

#include "../../paper_1002_3446_amd/csrc/bg_math.hpp"

int main() {
  uint64_t st = 0x9E3779B97F4A7C15ull;
  auto next = [&]() {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
  };
  for (int i = 0; i < 200000; ++i) {
    const uint64_t r = next();
    // uniform mantissa, exponent uniform in [-80, 40], plus values near 1
    double x;
    if (i % 4 == 0) {
      x = 1.0 + ((double)(int64_t)(r >> 11) - 0x1p52) * 0x1p-62;
    } else {
      const double m = 1.0 + (double)(r >> 12) * 0x1p-52;
      x = std::ldexp(m, (int)(r % 121) - 80);
    }
    std::printf("L %a %a\n", x, bgk::log_fp64(x));
  }
  const double edge[] = {0x1p-1074, 0x1p-1022, 0x1.fffffffffffffp1023, 1.0, 0.5, 2.0, 0.7071067811865476, 1.4142135623730951};
  for (double x : edge) std::printf("L %a %a\n", x, bgk::log_fp64(x));
  auto sc = [](double t) {
    double s, c;
    bgk::sincospi_fp64(t, &s, &c);
    std::printf("S %a %a %a\n", t, s, c);
  };
  for (int i = 0; i < 6000; ++i) {
    const uint64_t r = next();
    if (i % 3 == 0) {
      // within 2^-20 of a multiple of 1/4 (the reduction's switch points and the zeros)
      const double seam = 0.25 * (double)(r % 9);
      const double d = ((double)(int64_t)(next() >> 11) - 0x1p52) * 0x1p-72;
      sc(seam + d < 0.0 ? -(seam + d) : (seam + d > 2.0 ? 4.0 - (seam + d) : seam + d));
    } else {
      sc((double)((r >> 32) + 0.5) * 0x1p-31);  // t = 2 rho, rho = (u + 1/2) 2^-32
    }
  }
  for (int q = 0; q <= 8; ++q) sc(0.25 * q);
  return 0;
}
