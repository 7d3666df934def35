// Host-side reference: Philox4x32-10 blocks from the rocRAND library's
// engine, read from stdin as "c0 c1 c2 c3 k0 k1" (hex) and written as four hex
// words.  Used only to pin the oracle's generator to a library routine; the
// engine is placed at counter (c0,c1,c2,c3) through its public seek API
// (subsequence = c3:c2, offset = 4 * c1:c0, so c1 must stay below 2^30).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned a[6];
  while (std::scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
    unsigned long long seed = ((unsigned long long)a[5] << 32) | a[4];
    unsigned long long sub = ((unsigned long long)a[3] << 32) | a[2];
    unsigned long long off = 4ull * (((unsigned long long)a[1] << 32) | a[0]);
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 o = e.next4();
    std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
