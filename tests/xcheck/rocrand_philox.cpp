// Independent Philox4x32-10 source for cross-checking the oracle: rocRAND's
// header-only engine, used from host code only (no kernel, no HIP call).
// Reads lines "k0 k1 c0 c1 c2 c3" (hex) and prints the four output words.
// The engine takes key = seed, subsequence = counter words 2-3, and an offset
// counted in 32-bit outputs (4 per counter step, so c1 must stay below 2^30).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long step = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    rocrand_device::philox4x32_10_engine e(seed, subseq, 4ull * step);
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
