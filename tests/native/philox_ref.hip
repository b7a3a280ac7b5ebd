// Host-side driver for the oracle's Philox check: reads lines of six hexadecimal 32-bit
// words "c0 c1 c2 c3 k0 k1" (counter, key) from stdin and prints the four output words of
// Philox-4x32-10 for each, computed by the ROCm rocRAND library's own implementation of the
// published generator (an independent implementation, used here only as a reference).
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

struct Engine : rocrand_device::philox4x32_10_engine {
  uint4 words(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Engine e;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const uint4 r = e.words(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
