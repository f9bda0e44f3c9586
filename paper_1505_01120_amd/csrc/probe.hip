// Read-stream ceiling: the rate at which a plain kernel with nothing to do
// but read two float arrays (nontemporal float4 loads, four quads per array
// in flight per thread, grid-stride) streams from HBM on this GPU.  The bench
// reports the fused map-reduce against it beside the 8 TB/s peak.
//
// Built as its own library (libsparkcl_probe.so); it is a measurement tool,
// not part of the sparkcl API.
#include <hip/hip_runtime.h>

#include <cstdint>

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

} // namespace

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
