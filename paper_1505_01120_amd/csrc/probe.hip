// Measurement probes, built as their own library (libsparkcl_probe.so); they
// are measurement tools, not part of the sparkcl API.
//
// Read-stream ceiling: the rate at which a plain kernel with nothing to do
// but read two float arrays (nontemporal float4 loads, four quads per array
// in flight per thread, grid-stride) streams from HBM on this GPU.  The bench
// reports the fused map-reduce against it beside the 8 TB/s peak.
//
// VALU ceiling: register-only loops that issue nothing but vector ALU work,
// each thread on its own independent values, at full occupancy.  One runs
// the Monte-Carlo kernel's own Philox4x32-10 + quarter-disc loop body (the
// same device functions), the others a single instruction type each, so the
// issue rate of every instruction the Philox loop uses can be read off.
// Block 0's thread 0 also reads the shader-clock cycle counter and the
// constant-rate wall clock at its start and end, which gives the clock the
// loop actually ran at.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "philox_dev.h"
#include "sparkcl.h"

namespace {

constexpr int kThreads = 256;
constexpr int kQuads = 4; // quads per array in flight per thread

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const f4v gf4;

__device__ __forceinline__ f4v ld(const gf4 *p) { return __builtin_nontemporal_load(p); }

// Reads x[0..4 nq) and y[0..4 nq); nq is a multiple of kQuads * gridDim.x *
// kThreads, so every load is in bounds and every quad is read exactly once.
// Block b writes the sum of what it read to sink[b], so no load is dead.
__global__ __launch_bounds__(kThreads) void k_read_ceiling(const float *x, const float *y,
                                                           uint64_t nq, float *sink)
{
    const gf4 *X = (const gf4 *)x; // global address space
    const gf4 *Y = (const gf4 *)y;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    f4v s = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint64_t q = (uint64_t)blockIdx.x * kThreads + threadIdx.x; q < nq;
         q += kQuads * stride) {
        f4v a[kQuads], b[kQuads];
#pragma unroll
        for (int u = 0; u < kQuads; ++u) {
            a[u] = ld(X + q + u * stride);
            b[u] = ld(Y + q + u * stride);
        }
#pragma unroll
        for (int u = 0; u < kQuads; ++u)
            s += a[u] + b[u];
    }
    float v = s.x + s.y + s.z + s.w;
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o);
    __shared__ float w[kThreads / 64];
    if ((threadIdx.x & 63) == 0)
        w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = 0.0f;
        for (int i = 0; i < kThreads / 64; ++i)
            r += w[i];
        sink[blockIdx.x] = r;
    }
}

// ---- VALU ceiling ----------------------------------------------------------
enum ValuMix : uint32_t {
    MIX_PHILOX = 0,  // the Monte-Carlo loop body: one Philox block, two samples
    MIX_PHILOX2 = 1, // two independent Philox blocks per iteration
    MIX_XOR3 = 2,    // v_bitop3_b32 three-way xors, 8 independent chains
    MIX_MAD64 = 3,   // v_mad_u64_u32 32x32+64 -> 64, 8 independent chains
    MIX_ADD = 4,     // v_add_u32, 8 independent chains
    MIX_MULHI = 5,   // v_mul_hi_u32, 8 independent chains
    MIX_BITOP3_ADD = 6, // v_bitop3_b32 and v_add_u32 in turn, 8 chains of each
    MIX_MAD64_ADD = 7,  // v_mad_u64_u32 and v_add_u32 in turn, 8 chains of each
    MIX_COUNT = 8
};

__device__ __forceinline__ void clock_mark(uint64_t *clk, int at)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[2 * at] = clock64();
        clk[2 * at + 1] = wall_clock64();
    }
}

// Every thread runs `iters` iterations (four steps each for the single-
// instruction mixes) on values seeded from its global index; its result goes to sink[gid] so that no work is dead.
template <uint32_t MIX>
__global__ __launch_bounds__(kThreads) void k_valu(uint64_t seed, uint32_t pid, uint32_t iters,
                                                   uint32_t *sink, uint64_t *clk)
{
    clock_mark(clk, 0);
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t out = 0;
    if constexpr (MIX == MIX_PHILOX || MIX == MIX_PHILOX2) {
        // pair index p = gid + i * stride, as the tiles' threads stride over
        // their pairs
        const uint64_t stride = (uint64_t)gridDim.x * kThreads;
        uint64_t p = gid;
        uint32_t hits = 0;
        for (uint32_t i = 0; i < iters; ++i) {
            const sparkcl::U4 r =
                sparkcl::philox10(sparkcl::U4{(uint32_t)p, (uint32_t)(p >> 32), pid, 0u}, k0, k1);
            hits += sparkcl::disc_hit(r.x, r.y) + sparkcl::disc_hit(r.z, r.w);
            if constexpr (MIX == MIX_PHILOX2) {
                const uint64_t q = p + (uint64_t)iters * stride;
                const sparkcl::U4 t = sparkcl::philox10(
                    sparkcl::U4{(uint32_t)q, (uint32_t)(q >> 32), pid, 0u}, k0, k1);
                hits += sparkcl::disc_hit(t.x, t.y) + sparkcl::disc_hit(t.z, t.w);
            }
            p += stride;
        }
        out = hits;
    } else {
        uint32_t a[8];
        uint64_t w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] = gid * 0x9E3779B9u + (uint32_t)j * 0x7F4A7C15u + k0;
            w[j] = ((uint64_t)a[j] << 32) | (a[j] ^ k1);
        }
        for (uint32_t i = 0; i < iters; ++i) {
            // Four steps per iteration (the loop's scalar overhead is then a
            // small share of the issue slots).  Each step reads its chain and
            // the next one, so the compiler cannot fold a chain into a closed
            // form; all eight chains of a step are independent.
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const uint32_t s0 = k0 + (4 * i + st) * 0x85EBCA6Bu;
                uint32_t b[8];
                uint64_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    b[j] = a[j];
                    v[j] = w[j];
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if constexpr (MIX == MIX_XOR3)
                        a[j] = sparkcl::xor3(b[j], b[(j + 1) & 7], s0);
                    else if constexpr (MIX == MIX_MAD64)
                        w[j] = (uint64_t)(uint32_t)v[(j + 1) & 7] * s0 + v[j];
                    else if constexpr (MIX == MIX_ADD)
                        a[j] = b[j] + b[(j + 1) & 7];
                    else if constexpr (MIX == MIX_MULHI)
                        a[j] = __umulhi(b[j], b[(j + 1) & 7]);
                    else if constexpr (MIX == MIX_BITOP3_ADD) {
                        a[j] = sparkcl::xor3(b[j], b[(j + 1) & 7], s0);
                        w[j] = (uint32_t)v[j] + (uint32_t)v[(j + 1) & 7];
                    } else if constexpr (MIX == MIX_MAD64_ADD) {
                        w[j] = (uint64_t)(uint32_t)v[(j + 1) & 7] * s0 + v[j];
                        a[j] = b[j] + b[(j + 1) & 7];
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            out ^= a[j] ^ (uint32_t)w[j] ^ (uint32_t)(w[j] >> 32);
    }
    sink[gid] = out;
    clock_mark(clk, 1);
}

} // namespace

extern "C" __attribute__((visibility("default"))) int
sparkcl_probe_clock_rates(int device, uint32_t *peak_khz, uint32_t *wall_khz)
{
    // The device's peak shader clock and the constant rate of the wall clock
    // that the VALU probe's clock marks read (both in kHz).
    if (!peak_khz || !wall_khz)
        return SPARKCL_EINVAL;
    int a = 0, b = 0;
    if (hipDeviceGetAttribute(&a, hipDeviceAttributeClockRate, device) != hipSuccess ||
        hipDeviceGetAttribute(&b, hipDeviceAttributeWallClockRate, device) != hipSuccess)
        return SPARKCL_EHIP;
    *peak_khz = (uint32_t)a;
    *wall_khz = (uint32_t)b;
    return SPARKCL_OK;
}

extern "C" __attribute__((visibility("default"))) int
sparkcl_probe_valu(uint32_t mix, uint32_t grid, uint32_t iters, uint64_t seed, uint32_t pid,
                   uint32_t *sink, uint64_t *clk, void *stream)
{
    // One launch of the VALU probe `mix` (0 Philox loop, 1 two Philox blocks
    // per iteration, 2 xor3, 3 mad_u64_u32, 4 add_u32, 5 mul_hi_u32, 6 xor3
    // and add_u32, 7 mad_u64_u32 and add_u32) with
    // `grid` blocks of 256 threads, `iters` iterations per thread, on
    // `stream`.  sink: grid * 256 words (device); clk: 4 words (device),
    // receiving block 0's (shader clock, wall clock) at its start and its end.
    // A Philox probe covers pairs [0, grid * 256 * iters) (twice that for
    // mix 1) of partition `pid` under key `seed`, the same pairs a
    // Monte-Carlo partition of that many samples draws.  SPARKCL_EINVAL for
    // a bad argument, nothing launched.
    if (!sink || !clk || grid == 0 || grid > 65535u * 16u || iters == 0 || mix >= MIX_COUNT)
        return SPARKCL_EINVAL;
    if ((uintptr_t)sink & 3u || (uintptr_t)clk & 7u)
        return SPARKCL_EINVAL;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    switch (mix) {
    case MIX_PHILOX:
        hipLaunchKernelGGL(k_valu<MIX_PHILOX>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    case MIX_PHILOX2:
        hipLaunchKernelGGL(k_valu<MIX_PHILOX2>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    case MIX_XOR3:
        hipLaunchKernelGGL(k_valu<MIX_XOR3>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    case MIX_MAD64:
        hipLaunchKernelGGL(k_valu<MIX_MAD64>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    case MIX_ADD:
        hipLaunchKernelGGL(k_valu<MIX_ADD>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    case MIX_MULHI:
        hipLaunchKernelGGL(k_valu<MIX_MULHI>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    case MIX_BITOP3_ADD:
        hipLaunchKernelGGL(k_valu<MIX_BITOP3_ADD>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    default:
        hipLaunchKernelGGL(k_valu<MIX_MAD64_ADD>, dim3(grid), dim3(kThreads), 0, s, seed, pid, iters, sink, clk);
        break;
    }
    return hipGetLastError() == hipSuccess ? SPARKCL_OK : SPARKCL_EHIP;
}

extern "C" __attribute__((visibility("default"))) int
sparkcl_probe_read2(const float *x, const float *y, uint64_t n, uint32_t grid, float *sink,
                    void *stream)
{
    // One launch over x[0..n) and y[0..n) on `stream` (a hipStream_t; null is
    // the default stream) with `grid` blocks of 256 threads; sink receives
    // grid floats.  n must be a multiple of 4 * 4 * 256 * grid and x, y 16-byte
    // aligned device pointers; otherwise SPARKCL_EINVAL and nothing runs.
    if (!x || !y || !sink || grid == 0 || grid > 65535u * 16u)
        return SPARKCL_EINVAL;
    if ((((uintptr_t)x | (uintptr_t)y) & 15u) || (uintptr_t)sink & 3u)
        return SPARKCL_EINVAL;
    const uint64_t per_pass = 4ull * kQuads * kThreads * grid;
    if (n == 0 || n % per_pass)
        return SPARKCL_EINVAL;
    hipLaunchKernelGGL(k_read_ceiling, dim3(grid), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), x, y, n / 4, sink);
    return hipGetLastError() == hipSuccess ? SPARKCL_OK : SPARKCL_EHIP;
}
