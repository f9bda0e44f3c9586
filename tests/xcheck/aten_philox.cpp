// Independent Philox4x32-10 source for cross-checking the oracle: PyTorch's
// header-only at::philox_engine, compiled for the CPU.  Reads lines
// "k0 k1 c0 c1 c2 c3" (hex) and prints the four output words (hex).
// The engine takes key = seed, counter words 0-1 = offset, 2-3 = subsequence.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cinttypes>
#include <cstdio>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    at::philox_engine e(seed, subseq, offset);
    unsigned r0 = e(), r1 = e(), r2 = e(), r3 = e();
    std::printf("%08x %08x %08x %08x\n", r0, r1, r2, r3);
  }
  return 0;
}
