// Known-answer source for the oracle's Philox4x32-10: rocRAND's Philox engine,
// run on the host.  rocRAND keys the engine with seed = (k1 << 32) | k0, adds
// the subsequence to counter words (2, 3) and offset / 4 to words (0, 1); the
// first four outputs after construction are then Philox(counter, key).
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin, prints the four words.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (k1 << 32) | k0;
    unsigned long long subsequence = (c3 << 32) | c2;
    unsigned long long offset = 4ull * ((c1 << 32) | c0);
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
    uint4 r = eng.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
