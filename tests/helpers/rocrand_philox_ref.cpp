// Host-side reference for Philox4x32-10 taken from rocRAND's header-only
// engine (a library routine, independent of the oracle).  Reads lines
// "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the four output words.
// The engine's counter is set to (c0,c1,c2,c3) through rocrand_init with
// subsequence = c2 | c3 << 32 and offset = 4 * (c0 | c1 << 32); its key is
// the 64-bit seed (k0 low word, k1 high word).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long sub = c2 | (c3 << 32);
    unsigned long long off = 4ULL * (c0 | (c1 << 32));
    rocrand_init(seed, sub, off, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
