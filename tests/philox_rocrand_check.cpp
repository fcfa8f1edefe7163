// Black-box cross-check of the oracle's Philox4x32-10: reads lines
// "seed subsequence offset" and prints the four 32-bit words that rocRAND's
// open-source philox4x32_10 engine returns from that position.  Host code
// only; run by tests/test_oracle_philox.py.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine eng(seed, sub, off);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
