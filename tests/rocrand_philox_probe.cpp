// Host-only probe: prints Philox4x32-10 words from rocRAND's header-only engine for
// (seed, counter index n) pairs read from stdin, one "seed n" per line.  Used by the
// CPU tests as an independent implementation of the same generator.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned long long seed, n;
  while (std::scanf("%llu %llu", &seed, &n) == 2) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, 0ull, 4ull * n, &st);
    const uint4 w = rocrand4(&st);
    std::printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
  }
  return 0;
}
