// Independent Philox4x32-10 reference for the oracle's pin test: rocRAND's
// header-only engine, run on the host.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal)
// and prints the four output words of philox(counter, key).  The engine is
// positioned with key = k0 | k1 << 32, subsequence = c2 | c3 << 32 (the upper
// counter words) and offset = 4 * (c0 | c1 << 32) (the lower words, four outputs
// per block), so its current block is exactly the one for (c0, c1, c2, c3).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_device::philox4x32_10_engine e(k0 | (k1 << 32), c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)));
    unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
