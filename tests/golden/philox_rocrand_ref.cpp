// Reference stream from rocRAND's header-only Philox4x32-10 engine, used by the
// oracle tests as an independent implementation of Salmon et al. (SC'11).
// Prints the 4 output words for each counter given on stdin as
// "seed c0 c1 c2 c3" lines (the engine addresses a counter by
// subsequence = c2 + 2^32 c3 and offset = 4 (c0 + 2^32 c1)).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    unsigned long long sub = c2 | (c3 << 32);
    unsigned long long off = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 v = e.next4();
    std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
