// Philox4x32-10 and the quarter-disc hit test of the Monte-Carlo partition
// kernel (MapCLPartition, the SparkCLPi demo of paper sec. 3.2.1), as device
// functions.  The library's Monte-Carlo tiles and the VALU-ceiling probe
// (a register-only loop of the same instruction mix) both use them.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace sparkcl {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// The key words are wave-uniform and stay in scalar registers; each round is
// two 32x32->64 products and two three-way xors per lane.
struct U4 {
    uint32_t x, y, z, w;
};

// Three-way xor as one gfx950 v_bitop3_b32 (truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = xor3((uint32_t)(p1 >> 32), c.y, k0);
        n.y = (uint32_t)p1;
        n.z = xor3((uint32_t)(p0 >> 32), c.w, k1);
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Point (a, b) * 2^-24 from the top 24 bits of two words; a hit iff
// a^2 + b^2 <= 2^48, decided exactly in 64-bit integers (two 32x32->64
// multiply-adds).
__device__ __forceinline__ uint32_t disc_hit(uint32_t wa, uint32_t wb)
{
    const uint32_t a = wa >> 8, b = wb >> 8;
    const uint64_t r2 = (uint64_t)a * a + (uint64_t)b * b;
    return r2 <= (1ull << 48) ? 1u : 0u;
}

} // namespace sparkcl
