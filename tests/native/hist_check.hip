// Host-side driver for the exactness test of the library's fixed-point histogram sums:
// reads groups of hexadecimal doubles ("n x1 .. xn" per line), adds each group's values to
// fresh limbs with hist_split, normalises, and prints the rounded total (hex) per line.
#include <cstdio>
#include <cstdlib>

#include "../../paper_1002_3446_amd/csrc/bg_hist.hpp"

int main() {
  int n;
  while (std::scanf("%d", &n) == 1) {
    int64_t L[bgk::kHistLimbs] = {0};
    bool ok = true;
    for (int i = 0; i < n; ++i) {
      char buf[64];
      if (std::scanf("%63s", buf) != 1) return 1;
      const double x = std::strtod(buf, nullptr);
      ok = bgk::hist_split(x, [&](int j, int64_t c) { L[j] += c; }) && ok;
    }
    bgk::hist_normalise(L);
    std::printf("%s %a\n", ok ? "ok" : "rejected", bgk::hist_limbs_to_double(L));
  }
  return 0;
}
