// Host-side reference outputs of rocRAND's Philox4x32-10 engine, used to pin
// the CPU oracle's own Philox implementation.  Reads lines
// "c0 c1 c2 c3 k0 k1" (decimal) on stdin and prints the four output words
// for that counter and key.  The engine is positioned on a counter through
// its (seed, subsequence, offset) interface: seed = key, subsequence moves
// counter words 2-3, offset/4 moves counter words 0-1.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long subseq = c2 | (c3 << 32);
    unsigned long long offset = 4ULL * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
