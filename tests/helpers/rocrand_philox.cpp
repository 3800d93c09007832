// Prints rocRAND's Philox4x32-10 block for (counter, key) read from stdin,
// one "c0 c1 c2 c3 k0 k1" per line.  rocRAND keys the engine with the 64-bit
// seed (lo, hi), adds the subsequence to counter words (2, 3) and offset/4 to
// words (0, 1), so seed = k0 | k1 << 32, subsequence = c2 | c3 << 32 and
// an advance of c0 | c1 << 32 blocks select exactly the block at (counter, key).
// Host code only; used to pin the oracle's generator to an independent
// implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long X = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    rocrand_device::philox4x32_10_engine e(seed, sub, 0ULL);
    // advance the low counter words by X in pieces whose offsets fit 64 bits
    for (int i = 0; i < 4; i++) e.discard(4ULL * (X >> 2));
    e.discard(4ULL * (X & 3ULL));
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
