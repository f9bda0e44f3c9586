// HIP kernels of the SparkCL map -> reduce hot path, written for gfx950.
//
// A partition task (a MapCL / MapCLPartition / ReduceCL application, paper
// sec. 3.1.3) is cut into tiles of `tile_elems` elements.  One 256-thread
// block turns one tile into one partial:
//   1. streaming loop: coalesced 128-bit loads (float4), U quads per input
//      in flight per thread (2, 4 or 8, from the tuning table), the registry kernel's map applied per
//      element, each value added to a per-thread FP64 sum, a running max, or
//      a hit counter;
//   2. the per-thread values are combined across the wave with cross-lane
//      shuffles and across the block's waves through LDS in a fixed tree;
//   3. the partial is published and an arrival ticket taken; the block that
//      takes the last ticket combines the task's partials in FP64 in a fixed
//      order and writes the partition result (the tree-reduce of ReduceCL,
//      sec. 3.1.3 and 3.2.2); a task of one tile is finished by its block
//      directly.  The block that finishes the last task of a launch folds
//      the partition results into the RDD-level total.
// Tiles of at least one chunk (B threads x U quads, B the block size and U
// the quads each thread has in flight per input) deal a task's chunks
// round-robin to its tiles, so the tiles that run together read one sliding
// window of the task; smaller tiles are contiguous ranges.  Every element's
// owner thread and every combine order depend only on the tile size, the
// block size, U and x's 16-byte alignment, so results are identical run to
// run and across execution modes with the same tiles, block size and U.
//
// Compiled with -ffp-contract=off: the maps are the binary32 definition
// operation by operation.  No MFMA: nothing on this path is a contraction.

#include <hip/hip_runtime.h>

#include <cstddef>

#include "philox_dev.h"
#include "sparkcl_dev.h"

namespace sparkcl {

namespace {

constexpr float kNegInf = -__builtin_huge_valf();

__device__ __forceinline__ uint32_t uni(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ---- agent-scope atomics used by the last-block combine -----------------
__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_partial(Partial *p, double s, float m,
                                              uint64_t h, uint64_t n)
{
    uint64_t *w = reinterpret_cast<uint64_t *>(p);
    st_agent(w + 0, __double_as_longlong(s));
    st_agent(w + 1, (uint64_t)__float_as_uint(m));
    st_agent(w + 2, h);
    st_agent(w + 3, n);
}

__device__ __forceinline__ void load_partial(const Partial *p, double &s,
                                             float &m, uint64_t &h, uint64_t &n)
{
    const uint64_t *w = reinterpret_cast<const uint64_t *>(p);
    s = __longlong_as_double(ld_agent(w + 0));
    m = __uint_as_float((uint32_t)ld_agent(w + 1));
    h = ld_agent(w + 2);
    n = ld_agent(w + 3);
}

__device__ __forceinline__ uint64_t device_ns(uint32_t ns_per_tick)
{
    return (uint64_t)wall_clock64() * ns_per_tick;
}

// ---- streaming loads and stores -------------------------------------------
// The task's arrays arrive as generic pointers read from the task table; the
// casts below tell the compiler they are global memory, so it emits
// global_load/global_store instead of flat ones (flat accesses also count
// against the LDS/scalar counter and stall behind unrelated waits).  Every
// element is touched once, so the loads and stores are nontemporal.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const f4v gf4;
typedef __attribute__((address_space(1))) f4v gf4w;
typedef __attribute__((address_space(1))) const float gf1;
typedef __attribute__((address_space(1))) float gf1w;

__device__ __forceinline__ float4 ld4(const float *p)
{
    const f4v v = __builtin_nontemporal_load((gf4 *)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
// y and out need only 4-byte alignment: a 16-byte access at a 4-byte-aligned
// address is still one dwordx4 instruction (the memory pipeline splits it
// over the two 16-byte segments it touches), so arrays whose misalignments
// differ from x's stream as quads too.
typedef float f4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef __attribute__((address_space(1))) const f4a4 gf4u;
typedef __attribute__((address_space(1))) f4a4 gf4uw;
__device__ __forceinline__ float4 ld4u(const float *p)
{
    const f4a4 v = __builtin_nontemporal_load((gf4u *)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4u(float *p, const float4 &v)
{
    const f4a4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (gf4uw *)p);
}
__device__ __forceinline__ float ld1(const float *p)
{
    return __builtin_nontemporal_load((gf1 *)p);
}
__device__ __forceinline__ void st4(float *p, const float4 &v)
{
    const f4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (gf4w *)p);
}
__device__ __forceinline__ void st1(float *p, float v)
{
    __builtin_nontemporal_store(v, (gf1w *)p);
}

// Publication order without cache maintenance: the partials and results are
// written with agent-scope atomic stores, which write through the per-XCD L2
// to the device coherence point, and read back with agent-scope atomic loads,
// which bypass it.  Waiting for this thread's stores to complete before the
// arrival ticket is taken therefore makes them visible to the block that
// takes the last ticket, without the L2 write-back of a release fence (which
// costs half the streaming bandwidth when paid once per tile).
__device__ __forceinline__ void own_stores_complete()
{
    __builtin_amdgcn_s_waitcnt(0);
}

// ---- registry maps (one binary32 operation per step, in order) -----------
template <int D> struct PolyMap {
    static constexpr bool kTwo = false;
    static constexpr bool kGroup = false;
    float k[8];
    __device__ __forceinline__ float operator()(float x, float) const
    {
        float t = k[D];
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            float p = t * x;
            t = p + k[i];
        }
        return t;
    }
};

struct FmulMap {
    static constexpr bool kTwo = true;
    static constexpr bool kGroup = false;
    float c;
    __device__ __forceinline__ float operator()(float x, float y) const
    {
        float xy = x * y;
        float cx = c * x;
        return xy + cx;
    }
};

// Per-thread accumulator of one tile.  The sum is carried in FP64: on
// gfx950 a vector FP64 add issues at the full 32-bit rate, so converting and
// adding (two instructions) is cheaper than binary32 Neumaier compensation
// (seven), and a recursive FP64 sum of m terms is within (m-1) 2^-53 of the
// sum of magnitudes -- far inside the binary32 result's own resolution.
struct Acc {
    double s = 0.0;
    float m = kNegInf;
    uint32_t hits = 0;
    __device__ __forceinline__ void add(float v)
    {
        s += (double)v;
        m = fmaxf(m, v);
    }
};

// ---- elementwise tiles ------------------------------------------------------
// One quad of the map: four results, optionally stored, folded into the
// thread's accumulator in element order.
template <class M, bool W>
__device__ __forceinline__ void map_quad(const M &f, const float4 &xv,
                                         const float4 &yv, float *o, Acc &a)
{
    float4 v;
    v.x = f(xv.x, yv.x);
    v.y = f(xv.y, yv.y);
    v.z = f(xv.z, yv.z);
    v.w = f(xv.w, yv.w);
    if (W)
        st4u(o, v);
    a.add(v.x);
    a.add(v.y);
    a.add(v.z);
    a.add(v.w);
}

// Stream `ng` groups of the calling thread.  Group g is the U quads
// base(g) + u * B (u = 0..U-1, B the block size), in quads from x4/y4/o4: all the
// group's loads are issued, then the group is folded in order.  (Measured on
// MI355X: keeping a second group in flight while folding -- a register double
// buffer -- streams slower than this at every tile size and occupancy; the
// extra requests in flight cost more at the HBM than the overlap gains.)
//
// A map with run-time steps (kGroup: a fused chain) maps the whole group at
// once, so each step's uniform test and coefficient is paid once per group
// of 4 U elements per thread rather than once per element.
template <class M, bool W, int U, class Base>
__device__ __forceinline__ void stream_groups(const M &f, const float *x4,
                                              const float *y4, float *o4,
                                              uint64_t ng, Base base, Acc &a)
{
    const uint32_t B = blockDim.x;
    constexpr int NY = M::kTwo ? U : 1; // one-input maps carry no y buffer
    for (uint64_t g = 0; g < ng; ++g) {
        const uint64_t q0 = base(g);
        float4 xv[U], yv[NY];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xv[u] = ld4(x4 + 4 * (q0 + u * B));
            if (M::kTwo)
                yv[u] = ld4u(y4 + 4 * (q0 + u * B));
        }
        if constexpr (M::kGroup) {
            float v[4 * U];
            f.template group<U>(xv, M::kTwo ? yv : xv, v);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (W)
                    st4u(o4 + 4 * (q0 + u * B),
                         make_float4(v[4 * u], v[4 * u + 1], v[4 * u + 2], v[4 * u + 3]));
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    a.add(v[4 * u + e]);
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                map_quad<M, W>(f, xv[u], M::kTwo ? yv[u] : xv[u],
                               W ? o4 + 4 * (q0 + u * B) : nullptr, a);
        }
    }
}

// Scalar elements [i0, i1) of an elementwise task, strided over the block.
template <class M, bool W>
__device__ __forceinline__ void map_scalar(const M &f, const float *x,
                                           const float *y, float *out,
                                           uint64_t i0, uint64_t i1, Acc &a)
{
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        float v = f(ld1(x + i), M::kTwo ? ld1(y + i) : 0.0f);
        if (W)
            st1(out + i, v);
        a.add(v);
    }
}

// The scalar head of a task's range: the elements before x reaches a 16-byte
// boundary.  The quads after it are aligned for x; y and out, at any 4-byte
// alignment, are read and written with the same quad indices.
__device__ __forceinline__ uint32_t quad_head(const float *x, uint64_t n)
{
    const uint32_t mis = (uint32_t)(((uintptr_t)x & 15u) >> 2);
    return (uint32_t)min((uint64_t)((4u - mis) & 3u), n);
}

// Contiguous tile [begin, end): the middle in float4 quads (thread t owns
// quads t, t+B, t+2B, ...), the head before x's first 16-byte boundary and
// the ragged tail as single elements owned by threads 0..2.
template <class M, bool W, int U>
__device__ __forceinline__ void tile_contiguous(const M &f,
                                                const float *__restrict__ x,
                                                const float *__restrict__ y,
                                                float *__restrict__ out,
                                                uint64_t begin, uint64_t end,
                                                Acc &a)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t len = (uint32_t)(end - begin);
    const float *xb = x + begin;
    const float *yb = M::kTwo ? y + begin : nullptr;
    float *ob = W ? out + begin : nullptr;
    const uint32_t head = quad_head(xb, len);
    map_scalar<M, W>(f, xb, yb, ob, 0, head, a);

    const uint32_t B = blockDim.x;
    const uint32_t kStep = U * B;
    const uint32_t nq = (len - head) >> 2;
    const float *x4 = xb + head;
    const float *y4 = M::kTwo ? yb + head : nullptr;
    float *o4 = W ? ob + head : nullptr;
    // full groups of U quads owned by this thread
    const uint32_t full = (tid + (U - 1) * B < nq)
                              ? (nq - tid - (U - 1) * B + kStep - 1) / kStep
                              : 0u;
    stream_groups<M, W, U>(f, x4, y4, o4, full,
                           [&](uint64_t g) { return (uint64_t)tid + g * kStep; }, a);
    for (uint32_t q = tid + full * kStep; q < nq; q += B)
        map_quad<M, W>(f, ld4(x4 + 4u * q), M::kTwo ? ld4u(y4 + 4u * q) : float4{},
                       W ? o4 + 4u * q : nullptr, a);
    map_scalar<M, W>(f, xb, yb, ob, head + 4u * nq, len, a);
}

// Interleaved layout of a whole task (tiles of at least one chunk, 4 U B
// elements): the task's quad-aligned
// middle is cut into chunks of U * B quads, and tile j of nt owns
// chunks j, j + nt, j + 2 nt, ...; tile 0 also owns the unaligned head and
// the ragged tail.  Tiles that run at the same time (the queue hands out a
// task's tiles in order) then read neighbouring chunks, one sliding window
// per task instead of one stream per tile, which HBM serves at a higher rate.
// Returns the number of elements the tile covers.
template <class M, bool W, int U>
__device__ __forceinline__ uint64_t tile_interleaved(const M &f,
                                                     const float *__restrict__ x,
                                                     const float *__restrict__ y,
                                                     float *__restrict__ out,
                                                     uint64_t n, uint32_t head,
                                                     uint32_t nt, uint32_t j,
                                                     Acc &a)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t B = blockDim.x;
    const uint32_t kChunkQuads = U * B;
    const uint64_t nq = (n - head) >> 2;
    const uint64_t nfull = nq / kChunkQuads;
    const uint32_t rem = (uint32_t)(nq % kChunkQuads);
    const float *x4 = x + head;
    const float *y4 = M::kTwo ? y + head : nullptr;
    float *o4 = W ? out + head : nullptr;
    const uint64_t ng = nfull > j ? (nfull - j + nt - 1) / nt : 0;
    stream_groups<M, W, U>(f, x4, y4, o4, ng,
                           [&](uint64_t g) { return (j + g * nt) * kChunkQuads + tid; }, a);
    uint64_t count = 4 * ng * kChunkQuads;
    if (rem != 0 && nfull % nt == j) {
        const uint64_t q0 = nfull * kChunkQuads;
        for (uint32_t q = tid; q < rem; q += B)
            map_quad<M, W>(f, ld4(x4 + 4 * (q0 + q)),
                           M::kTwo ? ld4u(y4 + 4 * (q0 + q)) : float4{},
                           W ? o4 + 4 * (q0 + q) : nullptr, a);
        count += 4 * rem;
    }
    if (j == 0) {
        map_scalar<M, W>(f, x, y, out, 0, head, a);
        map_scalar<M, W>(f, x, y, out, head + 4 * nq, n, a);
        count += n - 4 * nq;
    }
    return count;
}

// Tile j of an elementwise task: interleaved when the tile size allows,
// else the contiguous range [jT, jT + T).  Returns the number of elements
// covered.
template <class M, bool W, int U>
__device__ __forceinline__ uint64_t tile_map(const M &f, const float *x,
                                             const float *y, float *out,
                                             uint64_t n, uint32_t T, uint32_t nt,
                                             uint32_t j, Acc &a)
{
    if (T >= 4u * U * blockDim.x)
        return tile_interleaved<M, W, U>(f, x, y, out, n, quad_head(x, n), nt, j, a);
    const uint64_t begin = (uint64_t)j * T;
    const uint64_t end = min(n, begin + T);
    if (begin < end)
        tile_contiguous<M, W, U>(f, x, y, out, begin, end, a);
    return begin < end ? end - begin : 0;
}

// MapCLPartition Monte-Carlo tile: samples [begin, end), begin even.  Pair p
// is the Philox block with counter (p lo, p hi, partition id, 0); sample 2p
// takes words (0, 1), sample 2p+1 words (2, 3).
__device__ __forceinline__ void tile_mc(uint64_t seed, uint32_t pid,
                                        uint64_t begin, uint64_t end, Acc &a)
{
    const uint64_t p0 = begin >> 1;
    const uint32_t npairs = (uint32_t)(((end + 1) >> 1) - p0);
    const bool odd_tail = (end & 1u) != 0;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t hits = 0;
    for (uint32_t i = threadIdx.x; i < npairs; i += blockDim.x) {
        const uint64_t p = p0 + i;
        const U4 r = philox10(U4{(uint32_t)p, (uint32_t)(p >> 32), pid, 0u}, k0, k1);
        const uint32_t second = (odd_tail && i == npairs - 1) ? 0u : 1u;
        hits += disc_hit(r.x, r.y) + (disc_hit(r.z, r.w) & second);
    }
    a.hits += hits;
}

// ---- wave and block combines --------------------------------------------
struct Red {
    double s;
    float m;
    uint64_t h, n;
};

__device__ __forceinline__ void wave_reduce(Red &r)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        r.s += __shfl_xor(r.s, o);
        r.m = fmaxf(r.m, __shfl_xor(r.m, o));
        r.h += __shfl_xor(r.h, o);
        r.n += __shfl_xor(r.n, o);
    }
}

// Block-wide combine; the result is valid in thread 0.  Waves are combined
// as a fixed pairwise tree ((w0 + w1) + (w2 + w3)) + ... over the block's
// B / 64 waves (4, 8 or 16).
__device__ __forceinline__ Red block_reduce(Red r)
{
    __shared__ double sh_s[kMaxWaves];
    __shared__ float sh_m[kMaxWaves];
    __shared__ uint64_t sh_h[kMaxWaves], sh_n[kMaxWaves];
    const uint32_t nw = blockDim.x >> 6;
    wave_reduce(r);
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh_s[w] = r.s;
        sh_m[w] = r.m;
        sh_h[w] = r.h;
        sh_n[w] = r.n;
    }
    __syncthreads();
    Red out = r;
    if (threadIdx.x == 0) {
        // in place in LDS (thread 0 alone): the pairwise tree over nw waves
        for (uint32_t step = 1; step < nw; step <<= 1)
            for (uint32_t i = 0; i + step < nw; i += 2 * step) {
                sh_s[i] = sh_s[i] + sh_s[i + step];
                sh_m[i] = fmaxf(sh_m[i], sh_m[i + step]);
                sh_h[i] += sh_h[i + step];
                sh_n[i] += sh_n[i + step];
            }
        out = Red{sh_s[0], sh_m[0], sh_h[0], sh_n[0]};
    }
    __syncthreads();
    return out;
}

// Fold the strided slice of `count` partials owned by this thread (in index
// order), then combine across the block.  Thread 0 holds the result.
template <class Load>
__device__ __forceinline__ Red combine_ordered(uint32_t count, Load load)
{
    Red r{0.0, kNegInf, 0, 0};
    for (uint32_t k = threadIdx.x; k < count; k += blockDim.x) {
        double s;
        float m;
        uint64_t h, n;
        load(k, s, m, h, n);
        r.s += s;
        r.m = fmaxf(r.m, m);
        r.h += h;
        r.n += n;
    }
    return block_reduce(r);
}

__device__ __forceinline__ void write_result(sparkcl_result *dst, uint32_t ops,
                                             const Red &r, uint64_t t_start,
                                             uint64_t t_done, int32_t status = SPARKCL_OK)
{
    sparkcl_result v;
    v.sum = (ops & SPARKCL_SUM) ? r.s : 0.0;
    v.max = (ops & SPARKCL_MAX) ? r.m : kNegInf;
    v.status = status;
    v.count = (ops & SPARKCL_COUNT) ? r.h : 0;
    v.n = r.n;
    v.t_arrive_ns = 0;
    v.t_admit_ns = 0;
    v.t_start_ns = t_start;
    v.t_done_ns = t_done;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(&v);
    uint64_t *d = reinterpret_cast<uint64_t *>(dst);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(v) / 8); ++i)
        st_agent(d + i, src[i]);
}

__device__ __forceinline__ void read_result(const sparkcl_result *p, double &s,
                                            float &m, uint64_t &h, uint64_t &n)
{
    const uint64_t *w = reinterpret_cast<const uint64_t *>(p);
    s = __longlong_as_double(ld_agent(w + 0));
    m = __uint_as_float((uint32_t)ld_agent(w + 1));
    h = ld_agent(w + 2);
    n = ld_agent(w + 3);
}

// ---- one tile, start to finish ------------------------------------------
// Thread 0 of the block that completes a task: write its result and, when
// serving, publish the completion word.  With `wait` false the result stores
// are left to complete while the block goes on: the persistent executor waits
// for all of a block's stores once, before the block counts itself out, and
// only then is any result read on the device (the RDD total).
__device__ __forceinline__ void finish_task(const TaskDev *__restrict__ tp, const LaunchOut &L,
                                            const Red &t, uint64_t t_start, uint32_t variant,
                                            uint32_t idx, bool wait = true)
{
    write_result(L.results + idx, uni(tp->ops), t, t_start, device_ns(L.ns_per_tick),
                 variant == V_DECLINED ? SPARKCL_EDECLINED : SPARKCL_OK);
    if (L.done) {
        // Serving: the result lives in host memory; publish it with a
        // system-scope release so the host sees the result before the word.
        __threadfence_system();
        __hip_atomic_store(L.done + idx, uni64(tp->seq) + 1, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    } else if (wait) {
        own_stores_complete();
    }
}

// Returns true in the block that completed the task (after writing its
// result); callers use it only for the RDD-level step.  kExec: called by the
// persistent executor, which waits for the result stores at its exit.
template <bool kExec = false, class Body>
__device__ __forceinline__ bool run_tile_with(const TaskDev *__restrict__ tp, uint32_t j,
                                              const LaunchOut &L, Body body)
{
    __shared__ uint32_t sh_last;
    TaskSync *__restrict__ sync = L.sync;
    const uint64_t t0 = device_ns(L.ns_per_tick);

    const uint32_t variant = uni(tp->variant);
    const uint32_t ntiles = uni(tp->ntiles);

    Acc a;
    const uint64_t count = body(a);

    Red r{a.s, a.m, a.hits, 0};
    r = block_reduce(r);

    const uint32_t idx = uni(tp->index);
    if (ntiles == 1) {
        // A task of one tile: its block finishes the task by construction,
        // so the partial, the start-time word and the arrival ticket (three
        // round trips to memory-side atomics) are skipped.  The ordered
        // combine of a single partial is the partial itself, except that its
        // FP64 sum starts from +0.0, which the + 0.0 below reproduces.
        if (threadIdx.x == 0)
            finish_task(tp, L, Red{r.s + 0.0, r.m, r.h, count}, t0, variant, idx, !kExec);
        __syncthreads();
        return true;
    }
    if (threadIdx.x == 0) {
        store_partial(tp->partials + j, r.s, r.m, r.h, count);
        // t_start keeps the bitwise complement of the earliest tile start, so
        // its cleared state (0) is the identity of the max below.
        __hip_atomic_fetch_max(&sync[idx].t_start, ~t0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        own_stores_complete();
        const uint32_t prev = __hip_atomic_fetch_add(&sync[idx].ticket, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        sh_last = (prev == ntiles - 1) ? 1u : 0u;
    }
    __syncthreads();
    // Every branch that guards a barrier must be provably uniform (a scalar
    // value): a condition read from LDS looks divergent to the compiler, and
    // its control-flow structurizer may then send some threads around a loop
    // latch without the others.
    const bool last = uni(sh_last) != 0;
    __syncthreads();
    if (!last)
        return false;

    // Last tile of the task: combine its partials in index order (agent-scope
    // atomic loads, issued only after the last ticket was observed).
    const Partial *parts = tp->partials;
    Red t = combine_ordered(ntiles, [&](uint32_t k, double &s, float &m,
                                        uint64_t &h, uint64_t &nn) {
        load_partial(parts + k, s, m, h, nn);
    });
    if (threadIdx.x == 0) {
        const uint64_t t_start = ~ld_agent(&sync[idx].t_start);
        __hip_atomic_store(&sync[idx].t_start, 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&sync[idx].ticket, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        finish_task(tp, L, t, t_start, variant, idx, !kExec);
    }
    // A barrier closes every thread-0 region that ends a loop iteration of the
    // callers: without it the compiler may sink the region past the loop
    // latch and let the other threads start the next iteration early.
    __syncthreads();
    return true;
}

// The registry kernels' tile body (maps fused with their reductions, or the
// Monte-Carlo count) run through the common tile epilogue.
template <bool kExec = false>
__device__ __forceinline__ bool run_tile(const TaskDev *__restrict__ tp, uint32_t j,
                                         const LaunchOut &L)
{
    return run_tile_with<kExec>(tp, j, L, [&](Acc &a) -> uint64_t {
        const uint32_t variant = uni(tp->variant);
        const uint32_t T = uni(tp->tile_elems);
        const uint32_t ntiles = uni(tp->ntiles);
        const uint64_t n = uni64(tp->n);
        uint64_t count = 0;
        const float *x = tp->in0;
        const float *y = tp->in1;
        float *o = tp->out;
        const uint32_t U = uni(tp->unroll);
        // the tile loop for map f with U quads in flight per thread
#define SPARKCL_TILE_U(MAP, WR, f)                                             \
    (U == 2   ? tile_map<MAP, WR, 2>(f, x, y, o, n, T, ntiles, j, a)               \
     : U == 8 ? tile_map<MAP, WR, 8>(f, x, y, o, n, T, ntiles, j, a)               \
              : tile_map<MAP, WR, 4>(f, x, y, o, n, T, ntiles, j, a))
        if (variant < V_FMUL) {
            const bool w = variant >= V_POLYW;
            const uint32_t d = variant & 7u;
            float k[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                k[i] = tp->coef[i];
#define SPARKCL_POLY_CASE(D)                                                   \
        case D: {                                                                  \
            PolyMap<D> f;                                                          \
            for (int i = 0; i < 8; ++i)                                            \
                f.k[i] = k[i];                                                     \
            count = w ? SPARKCL_TILE_U(PolyMap<D>, true, f)                        \
                      : SPARKCL_TILE_U(PolyMap<D>, false, f);                      \
        } break;
            switch (d) {
                SPARKCL_POLY_CASE(0)
                SPARKCL_POLY_CASE(1)
                SPARKCL_POLY_CASE(2)
                SPARKCL_POLY_CASE(3)
                SPARKCL_POLY_CASE(4)
                SPARKCL_POLY_CASE(5)
                SPARKCL_POLY_CASE(6)
                SPARKCL_POLY_CASE(7)
            }
#undef SPARKCL_POLY_CASE
        } else if (variant == V_FMUL || variant == V_FMULW) {
            FmulMap f{tp->c};
            count = variant == V_FMULW ? SPARKCL_TILE_U(FmulMap, true, f)
                                       : SPARKCL_TILE_U(FmulMap, false, f);
        } else if (variant == V_MC) {
            const uint64_t begin = (uint64_t)j * T;
            const uint64_t end = min(n, begin + T);
            if (begin < end) {
                tile_mc(uni64(tp->seed), uni(tp->pid), begin, end, a);
                count = end - begin;
            }
        } // V_DECLINED: nothing to do; the empty partial leaves the total as is
#undef SPARKCL_TILE_U
        return count;
    });
}

// The RDD-level total: all partition results folded in task order (run by
// one block once every task of the launch has its result).
__device__ __forceinline__ void rdd_total(const LaunchOut &L)
{
    const sparkcl_result *res = L.results;
    Red t = combine_ordered(L.ntasks, [&](uint32_t k, double &s, float &m,
                                          uint64_t &h, uint64_t &n) {
        read_result(res + k, s, m, h, n);
    });
    if (threadIdx.x == 0 && L.total) {
        write_result(L.total, SPARKCL_SUM | SPARKCL_MAX | SPARKCL_COUNT, t, 0,
                     device_ns(L.ns_per_tick));
        own_stores_complete();
    }
    __syncthreads();
}

// RDD-level step of the per-partition launches, run by the block that
// completed a task: the block that completes the last task of the sequence
// folds all partition results.
__device__ __forceinline__ void rdd_step(const LaunchOut &L)
{
    __shared__ uint32_t sh_last;
    if (L.ntasks == 0)
        return;
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(&L.ctl->rdd_ticket, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        sh_last = (prev == L.ntasks - 1) ? 1u : 0u;
    }
    __syncthreads();
    const bool last = uni(sh_last) != 0;
    __syncthreads();
    if (!last)
        return;
    rdd_total(L);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&L.ctl->rdd_ticket, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        own_stores_complete();
    }
    __syncthreads();
}

// ---- fused map chains ------------------------------------------------------
// A task's registry map followed by up to kMaxPost POLY stages on the running
// binary32 value (map -> map -> ... -> reduce in one pass).  Every Horner step
// is one binary32 multiply and one add in the written order.  Degrees are
// run-time values: a stage's eight coefficients are loaded (scalar loads from
// the uniform task or chain table) into registers at the stage's start, and
// its steps are unrolled to degree 7, each taken under a uniform test, so the
// coefficients are indexed by constants and the tests cost one scalar branch
// per group of values.

// t[e] <- p(x[e]) for the degree-d polynomial with coefficients kp[0..d].
template <int NV>
__device__ __forceinline__ void horner_group(const float *__restrict__ kp, uint32_t d,
                                             const float *x, float *t)
{
    float k[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        k[i] = kp[i];
    float top = k[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        top = d == (uint32_t)i ? k[i] : top;
#pragma unroll
    for (int e = 0; e < NV; ++e)
        t[e] = top;
#pragma unroll
    for (int i = 6; i >= 0; --i) {
        if ((uint32_t)i < d) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const float p = t[e] * x[e];
                t[e] = p + k[i];
            }
        }
    }
}

template <bool TWO> struct ChainMap {
    static constexpr bool kTwo = TWO;
    static constexpr bool kGroup = true;
    const float *k0; // the task's own POLY coefficients
    uint32_t d0;
    float c;
    const ChainDev *ch;
    uint32_t npost;

    // v[0..NV) <- the chain over x[0..NV) (and y), in element order
    template <int NV>
    __device__ __forceinline__ void apply(float *x, const float *y, float *v) const
    {
        if (TWO) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const float xy = x[e] * y[e];
                const float cx = c * x[e];
                v[e] = xy + cx;
            }
        } else {
            horner_group<NV>(k0, d0, x, v);
        }
        for (uint32_t s = 0; s < npost; ++s) {
#pragma unroll
            for (int e = 0; e < NV; ++e)
                x[e] = v[e];
            horner_group<NV>(ch->coef[s], uni(ch->deg[s]), x, v);
        }
    }
    template <int U>
    __device__ __forceinline__ void group(const float4 *xv, const float4 *yv, float *v) const
    {
        constexpr int NV = 4 * U;
        float x[NV], y[TWO ? NV : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x[4 * u] = xv[u].x;
            x[4 * u + 1] = xv[u].y;
            x[4 * u + 2] = xv[u].z;
            x[4 * u + 3] = xv[u].w;
            if (TWO) {
                y[4 * u] = yv[u].x;
                y[4 * u + 1] = yv[u].y;
                y[4 * u + 2] = yv[u].z;
                y[4 * u + 3] = yv[u].w;
            }
        }
        apply<NV>(x, y, v);
    }
    __device__ __forceinline__ float operator()(float x, float y) const
    {
        float v;
        apply<1>(&x, &y, &v);
        return v;
    }
};

template <bool TWO>
__device__ __forceinline__ ChainMap<TWO> chain_map(const TaskDev *tp, const ChainDev *ch)
{
    return ChainMap<TWO>{tp->coef, uni(tp->variant) & 7u, tp->c, ch, uni(ch->npost)};
}

// Tile j of a task with a map chain, through the common tile epilogue.
template <int UC>
__device__ __forceinline__ bool chain_tile(const TaskDev *__restrict__ tp,
                                           const ChainDev *__restrict__ chain, uint32_t j,
                                           const LaunchOut &L)
{
    return run_tile_with<true>(tp, j, L, [&](Acc &a) -> uint64_t {
        const uint32_t variant = uni(tp->variant);
        if (variant == V_DECLINED)
            return 0;
        const uint32_t T = uni(tp->tile_elems);
        const uint32_t nt = uni(tp->ntiles);
        const uint64_t n = uni64(tp->n);
        const float *x = tp->in0;
        const float *y = tp->in1;
        float *o = tp->out;
        const bool two = variant == V_FMUL || variant == V_FMULW;
        const bool w = variant == V_FMULW || (variant >= V_POLYW && variant < V_FMUL);
        if (two) {
            const ChainMap<true> f = chain_map<true>(tp, chain);
            return w ? tile_map<ChainMap<true>, true, UC>(f, x, y, o, n, T, nt, j, a)
                     : tile_map<ChainMap<true>, false, UC>(f, x, y, o, n, T, nt, j, a);
        }
        const ChainMap<false> f = chain_map<false>(tp, chain);
        return w ? tile_map<ChainMap<false>, true, UC>(f, x, y, o, n, T, nt, j, a)
                 : tile_map<ChainMap<false>, false, UC>(f, x, y, o, n, T, nt, j, a);
    });
}

// ---- kernels --------------------------------------------------------------

// One partition per launch: blocks stride over the task's tiles.
__global__ __launch_bounds__(kMaxBlock) void k_task(const TaskDev *__restrict__ task,
                                                 LaunchOut L)
{
    const uint32_t ntiles = uni(task->ntiles);
    for (uint32_t j = blockIdx.x; j < ntiles; j += gridDim.x)
        if (run_tile(task, j, L))
            rdd_step(L);
}

// Persistent executor: a fixed grid of blocks takes tiles from the queue with
// one atomic each until the queue is empty; thread 0 asks for the next tile
// while the current one streams, so the queue round trip is hidden.  The last
// block to leave resets the queue head, so the next launch of the same plan
// needs no clearing.
template <class Tile>
__device__ __forceinline__ void executor(const TaskDev *__restrict__ tasks,
                                         const TileRef *__restrict__ tiles, uint32_t ntiles,
                                         const LaunchOut &L, Tile tile)
{
    __shared__ uint32_t sh_tile;
    if (threadIdx.x == 0)
        sh_tile = __hip_atomic_fetch_add(&L.ctl->head, 1u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    uint32_t t = uni(sh_tile);
    __syncthreads();
    while (t < ntiles) {
        uint32_t next = 0;
        if (threadIdx.x == 0)
            next = __hip_atomic_fetch_add(&L.ctl->head, 1u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        const TileRef tr = tiles[t];
        const TaskDev *tp = tasks + uni(tr.task);
        tile(tp, uni(tr.tile));
        if (threadIdx.x == 0)
            sh_tile = next;
        __syncthreads();
        t = uni(sh_tile);
        __syncthreads();
    }
    // The last block to leave has every task's result (each block waited for
    // its own stores before it counted itself out): it folds the RDD total,
    // once per launch instead of one contended ticket per task, and resets
    // the queue for the next launch.
    __shared__ uint32_t sh_out;
    if (threadIdx.x == 0) {
        own_stores_complete();
        sh_out = __hip_atomic_fetch_add(&L.ctl->exited, 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1
                     ? 1u
                     : 0u;
    }
    __syncthreads();
    if (uni(sh_out) != 0) {
        if (L.ntasks != 0)
            rdd_total(L);
        if (threadIdx.x == 0) {
            __hip_atomic_store(&L.ctl->head, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&L.ctl->exited, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ __launch_bounds__(kMaxBlock) void k_batch(const TaskDev *__restrict__ tasks,
                                                  const TileRef *__restrict__ tiles,
                                                  uint32_t ntiles, LaunchOut L)
{
    executor(tasks, tiles, ntiles, L,
             [&](const TaskDev *tp, uint32_t j) { return run_tile<true>(tp, j, L); });
}

// The persistent executor for batches whose tasks are all Monte-Carlo ones:
// the same queue and tile epilogue around the Philox tile body alone.  The
// streaming bodies set k_batch's register count (and so its waves per CU);
// without them this kernel holds half the registers and fits twice the
// waves, which the VALU-bound loop needs to issue near its rate (measured on
// MI355X: 0.95 wave-instructions per CU per clock at 3 blocks per CU, 1.04
// at 8).  A declined task (empty partial) runs no body.
__global__ __launch_bounds__(kMaxBlock) void k_batch_mc(const TaskDev *__restrict__ tasks,
                                                     const TileRef *__restrict__ tiles,
                                                     uint32_t ntiles, LaunchOut L)
{
    executor(tasks, tiles, ntiles, L, [&](const TaskDev *tp, uint32_t j) {
        return run_tile_with<true>(tp, j, L, [&](Acc &a) -> uint64_t {
            if (uni(tp->variant) != V_MC)
                return 0;
            const uint32_t T = uni(tp->tile_elems);
            const uint64_t n = uni64(tp->n);
            const uint64_t begin = (uint64_t)j * T;
            const uint64_t end = min(n, begin + T);
            if (begin >= end)
                return 0;
            tile_mc(uni64(tp->seed), uni(tp->pid), begin, end, a);
            return end - begin;
        });
    });
}

// The persistent executor over tasks that share one map chain, with UC float4
// loads in flight per thread and input (4, or 8 for short chains run at one
// block per CU, where the deeper stream hides the Horner steps' latency that
// more blocks would otherwise have to).
template <int UC>
__global__ __launch_bounds__(kBlock) void k_chain(const TaskDev *__restrict__ tasks,
                                                  const TileRef *__restrict__ tiles,
                                                  uint32_t ntiles,
                                                  const ChainDev *__restrict__ chain,
                                                  LaunchOut L)
{
    executor(tasks, tiles, ntiles, L,
             [&](const TaskDev *tp, uint32_t j) { return chain_tile<UC>(tp, chain, j, L); });
}

// MapCL materialisation only (no reduction): out[i] = map(x[i] [, y[i]]),
// grid-stride over float4 quads when the arrays share their alignment.
template <class M>
__device__ __forceinline__ void map_only(const M &f, const float *__restrict__ x,
                                         const float *__restrict__ y,
                                         float *__restrict__ out, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t head = quad_head(x, n);
    for (uint64_t i = gtid; i < head; i += stride)
        st1(out + i, f(ld1(x + i), M::kTwo ? ld1(y + i) : 0.0f));
    const uint64_t nq = (n - head) >> 2;
    const float *x4 = x + head;
    const float *y4 = M::kTwo ? y + head : nullptr;
    float *o4 = out + head;
    for (uint64_t q = gtid; q < nq; q += stride) {
        const float4 xv = ld4(x4 + 4 * q);
        const float4 yv = M::kTwo ? ld4u(y4 + 4 * q) : xv;
        float4 v;
        v.x = f(xv.x, yv.x);
        v.y = f(xv.y, yv.y);
        v.z = f(xv.z, yv.z);
        v.w = f(xv.w, yv.w);
        st4u(o4 + 4 * q, v);
    }
    const uint64_t t0 = head + 4 * nq;
    if (gtid < n - t0)
        st1(out + t0 + gtid, f(ld1(x + t0 + gtid), M::kTwo ? ld1(y + t0 + gtid) : 0.0f));
}

__global__ __launch_bounds__(kBlock) void k_map(const TaskDev *__restrict__ tp,
                                                uint64_t n, uint32_t variant)
{
    const float *x = tp->in0;
    const float *y = tp->in1;
    float *o = tp->out;
    if (variant < V_FMUL) {
        float k[8];
        for (int i = 0; i < 8; ++i)
            k[i] = tp->coef[i];
#define SPARKCL_MAP_CASE(D)                                                    \
    case D: {                                                                  \
        PolyMap<D> f;                                                          \
        for (int i = 0; i < 8; ++i)                                            \
            f.k[i] = k[i];                                                     \
        map_only(f, x, y, o, n);                                               \
    } break;
        switch (variant & 7u) {
            SPARKCL_MAP_CASE(0)
            SPARKCL_MAP_CASE(1)
            SPARKCL_MAP_CASE(2)
            SPARKCL_MAP_CASE(3)
            SPARKCL_MAP_CASE(4)
            SPARKCL_MAP_CASE(5)
            SPARKCL_MAP_CASE(6)
            SPARKCL_MAP_CASE(7)
        }
#undef SPARKCL_MAP_CASE
    } else {
        FmulMap f{tp->c};
        map_only(f, x, y, o, n);
    }
}

// Clears library workspaces with a kernel (no memset nodes in captured work).
// ---- array-valued ReduceCL ----------------------------------------------------
// The RDD's elements are float arrays of one length; the two-input combiner
// (Fig 3 adds two arrays elementwise) folds them pairwise along a fixed
// tree: over elements [k0, k1) the tree splits at k0 + the largest power of
// two below the count, left part first.  Each thread owns V columns and
// walks the leaves in order with a binary counter of partial results: slot j
// holds the finished perfect subtree of 2^j leaves, a new leaf merges with
// the full slots of the counter's carry chain, and at the end the occupied
// slots are merged from the smallest (rightmost) up.  That is exactly the
// tree above, so every position sees the same sequence of binary32
// combines as the definition.  Eight aligned leaves are combined as a perfect
// tree first and enter the counter at level 3.
//
// A pass reduces chunks of S leaves (S a power of two unless the pass has a
// single chunk); chunk c writes its tree to row c of the output.  Full chunks
// are aligned perfect subtrees and the last chunk is the tree of the
// remaining suffix, so a later pass over the chunk rows, with the same rule,
// rebuilds the tree over all elements.
constexpr int kTreeSlots = 13; // up to 2^12 leaves per chunk

template <int V> struct TreeVec;
template <> struct TreeVec<1> {
    typedef float T;
    static __device__ __forceinline__ T ld(const float *p) { return ld1(p); }
    static __device__ __forceinline__ void st(float *p, T v) { st1(p, v); }
};
template <> struct TreeVec<4> {
    typedef float4 T;
    static __device__ __forceinline__ T ld(const float *p) { return ld4u(p); }
    static __device__ __forceinline__ void st(float *p, T v) { st4u(p, v); }
};

template <uint32_t COMB>
__device__ __forceinline__ float comb1(float a, float b)
{
    if (COMB == SPARKCL_VADD)
        return a + b;
    return (b > a) ? b : a;
}
template <uint32_t COMB>
__device__ __forceinline__ float comb(float a, float b)
{
    return comb1<COMB>(a, b);
}
template <uint32_t COMB>
__device__ __forceinline__ float4 comb(const float4 &a, const float4 &b)
{
    return make_float4(comb1<COMB>(a.x, b.x), comb1<COMB>(a.y, b.y),
                       comb1<COMB>(a.z, b.z), comb1<COMB>(a.w, b.w));
}

// Insert a perfect subtree of 2^L leaves that starts at leaf `pos` (a
// multiple of 2^L) into the counter.  `pos` is wave-uniform, so every branch
// here is a scalar branch and every slot index is a compile-time constant.
template <int L, uint32_t COMB, class T>
__device__ __forceinline__ void tree_insert(T (&slot)[kTreeSlots], uint32_t pos, T v)
{
    // the carry chain: the full slots L, L+1, ... below the first empty one
    const uint32_t full = (uint32_t)__builtin_ctz(~(pos >> L));
#pragma unroll
    for (int j = L; j < kTreeSlots; ++j) {
        if ((uint32_t)j < L + full)
            v = comb<COMB>(slot[j], v);
        else if ((uint32_t)j == L + full)
            slot[j] = v;
    }
}

template <int V, uint32_t COMB>
__global__ __launch_bounds__(kBlock) void k_tree(TreeArgs a)
{
    typedef TreeVec<V> TV;
    typedef typename TV::T T;
    const uint64_t col = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * V;
    if (col >= a.len)
        return; // no barriers below
    const uint32_t c = blockIdx.y;
    const uint32_t k0 = c * a.chunk;
    const uint32_t m = min(a.count - k0, a.chunk);
    auto leaf = [&](uint32_t i) -> const float * {
        const uint32_t kk = k0 + i;
        return (a.ptrs ? a.ptrs[kk] : a.base + (uint64_t)kk * a.stride) + col;
    };
    T slot[kTreeSlots];
    uint32_t i = 0;
    for (; i + 8 <= m; i += 8) {
        T v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            v[b] = TV::ld(leaf(i + b));
        const T l = comb<COMB>(comb<COMB>(v[0], v[1]), comb<COMB>(v[2], v[3]));
        const T r = comb<COMB>(comb<COMB>(v[4], v[5]), comb<COMB>(v[6], v[7]));
        tree_insert<3, COMB>(slot, i, comb<COMB>(l, r));
    }
    for (; i < m; ++i)
        tree_insert<0, COMB>(slot, i, TV::ld(leaf(i)));
    // merge the occupied slots, smallest (rightmost) first
    T acc{};
    bool have = false;
#pragma unroll
    for (int j = 0; j < kTreeSlots; ++j) {
        if (m & (1u << j)) {
            acc = have ? comb<COMB>(slot[j], acc) : slot[j];
            have = true;
        }
    }
    TV::st(a.out + (uint64_t)c * a.len + col, acc);
}

// Wide variant (float4 columns only): a thread owns CPT float4 columns BT
// quads apart, so a block of BT threads reads CPT * BT * 16 bytes of one leaf
// contiguously, and the leaves are walked two at a time: each pair is a
// perfect subtree that enters the counter at level 1.  Fewer leaves and
// longer runs of each leaf in flight keep the HBM row buffers open (measured
// on MI355X over 64 arrays of 2^22 floats: 32 KiB per leaf per block, as 512
// threads of 4 columns, streams at 6.7 TB/s; 16 KiB per leaf per block in
// 256 threads at 6.4; eight leaves of 4 KiB at 5.3).  The counter holds
// kTreeWideSlots levels per column, so a chunk has at most 64 leaves.
constexpr int kTreeWideSlots = 7;
static_assert(kTreeWideChunk == 1u << (kTreeWideSlots - 1), "chunk fits the counter");

template <int L, uint32_t COMB, int CPT>
__device__ __forceinline__ void tree_insert_cols(float4 (&slot)[kTreeWideSlots][CPT],
                                                 uint32_t pos, float4 (&v)[CPT])
{
    const uint32_t full = (uint32_t)__builtin_ctz(~(pos >> L));
#pragma unroll
    for (int j = L; j < kTreeWideSlots; ++j) {
        if ((uint32_t)j < L + full) {
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                v[c] = comb<COMB>(slot[j][c], v[c]);
        } else if ((uint32_t)j == L + full) {
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                slot[j][c] = v[c];
        }
    }
}

template <uint32_t COMB, int CPT, int BT>
__global__ __launch_bounds__(BT) void k_tree_wide(TreeArgs a)
{
    const uint64_t nq = a.len >> 2;
    const uint64_t q0 = (uint64_t)blockIdx.x * BT * CPT + threadIdx.x;
    if (q0 >= nq)
        return; // no barriers below
    bool ok[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c)
        ok[c] = q0 + (uint64_t)c * BT < nq;
    const uint32_t ch = blockIdx.y;
    const uint32_t k0 = ch * a.chunk;
    const uint32_t m = min(a.count - k0, a.chunk);
    auto leaf = [&](uint32_t i) -> const float * {
        const uint32_t kk = k0 + i;
        return (a.ptrs ? a.ptrs[kk] : a.base + (uint64_t)kk * a.stride) + 4 * q0;
    };
    auto load = [&](uint32_t i, float4 (&v)[CPT]) {
        const float *p = leaf(i);
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            v[c] = ok[c] ? ld4u(p + 4 * (uint64_t)c * BT) : float4{};
    };
    float4 slot[kTreeWideSlots][CPT];
    uint32_t i = 0;
    for (; i + 2 <= m; i += 2) {
        float4 l[CPT], r[CPT];
        load(i, l);
        load(i + 1, r);
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            l[c] = comb<COMB>(l[c], r[c]);
        tree_insert_cols<1, COMB, CPT>(slot, i, l);
    }
    if (i < m) {
        float4 v[CPT];
        load(i, v);
        tree_insert_cols<0, COMB, CPT>(slot, i, v);
    }
    float4 acc[CPT];
    bool have = false;
#pragma unroll
    for (int j = 0; j < kTreeWideSlots; ++j) {
        if (m & (1u << j)) {
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                acc[c] = have ? comb<COMB>(slot[j][c], acc[c]) : slot[j][c];
            have = true;
        }
    }
    float *o = a.out + (uint64_t)ch * a.len + 4 * q0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
        if (ok[c])
            st4u(o + 4 * (uint64_t)c * BT, acc[c]);
}

__global__ __launch_bounds__(kBlock) void k_zero(uint32_t *p, uint64_t words)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += stride)
        p[i] = 0u;
}

// ---- WordCount --------------------------------------------------------------
// The word-count demo (sec. 3.2.3) as a partition kernel over a byte stream:
// a word is a maximal run of non-whitespace bytes, counted under the 64-bit
// FNV-1a hash of its bytes (Fowler, Noll, Vo: xor the byte in, multiply by
// the 64-bit FNV prime).  Blocks stage 4 KiB chunks of text (plus a 256-byte
// look-ahead) in LDS; the thread owning a word's first byte hashes it and
// counts it in the block's LDS hash table (the paper's "local data"), which
// absorbs the frequent words of a skewed vocabulary.  Words that find no
// LDS slot within a few probes are appended to the block's spill region of
// their key's partition (a plain store at an LDS-counted position); a merge
// kernel then counts each partition's spilled keys in LDS and adds each
// distinct key once to the global open-addressing table.  (Adding every such word to the global table
// with a device-scope atomic, as a first version did, cost more than the
// scan: those atomics are carried out at the memory side, one round trip
// each.)  The LDS tables themselves, and the words that overflow a spill
// region, go to the table with atomics.  Counts are integers, so the result
// does not depend on which block counts which word.
constexpr uint32_t kWcChunk = 4096;   // bytes per chunk: 16 per thread
constexpr uint32_t kWcLook = 256;     // look-ahead bytes staged after a chunk
constexpr uint32_t kWcSlots = 2048;   // LDS hash slots per block
constexpr uint32_t kWcProbes = 2;     // LDS probes before a word spills
static_assert(kWcChunk == 16 * kBlock, "one 16-byte span per thread");

__device__ __forceinline__ bool wc_space(uint32_t b)
{
    return b == 0x20u || (b - 0x09u) <= 4u; // space, tab, LF, VT, FF, CR
}

__device__ __forceinline__ uint64_t fnv_step(uint64_t h, uint32_t b)
{
    return (h ^ (uint64_t)b) * 1099511628211ull;
}

// Add c to key h in the global table (keys 0 = empty; a word whose hash is 0
// is counted in ctl[1] instead).
__device__ void wc_global_add(const WcArgs &a, uint64_t h, uint64_t c)
{
    if (h == 0) {
        atomicAdd((unsigned long long *)&a.ctl[1], (unsigned long long)c);
        return;
    }
    // Probe sequences are bounded: at the load factor of 1/2 that a table
    // within capacity keeps, a run of 2^16 occupied slots does not happen, so
    // only an overflowing table reaches the bound.  Every 64 probes the
    // table-full flag is checked, so once the table is full the remaining
    // words stop early (the call fails with ETOOBIG).
    uint64_t s = h & a.mask;
    const uint64_t probes = min(a.mask, (uint64_t)0xFFFF);
    for (uint64_t probe = 0; probe <= probes; ++probe) {
        if ((probe & 63) == 63 &&
            __hip_atomic_load(&a.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        const uint64_t k = a.keys[s];
        if (k == h) {
            atomicAdd((unsigned long long *)&a.counts[s], (unsigned long long)c);
            return;
        }
        if (k == 0) {
            const uint64_t old =
                atomicCAS((unsigned long long *)&a.keys[s], 0ull, (unsigned long long)h);
            if (old == 0 || old == h) {
                atomicAdd((unsigned long long *)&a.counts[s], (unsigned long long)c);
                return;
            }
        }
        s = (s + 1) & a.mask;
    }
    atomicOr((unsigned long long *)&a.ctl[2], 1ull); // table full
}

// The LDS counts are 32-bit: a block counts at most one word per two bytes
// of the text it scans, and a block scans either one 4 KiB chunk or at most
// 1/256 of the text (a grid of at least one block per CU), which is limited
// to 2^40 bytes.
// A word that found no LDS slot: appended to this block's spill region of
// its partition, or, when the region is full (or there are none, or its key
// is 0), added to the table directly.  scnt: the block's per-partition
// append counters in LDS.
__device__ __forceinline__ void wc_spill(uint32_t *scnt, const WcArgs &a, uint64_t h)
{
    if (a.spill_cap != 0 && h != 0) {
        const uint32_t p = (uint32_t)(h >> (64 - kWcPartBits));
        const uint32_t pos = atomicAdd(&scnt[p], 1u);
        if (pos < a.spill_cap) {
            a.spill[((uint64_t)blockIdx.x << kWcPartBits | p) * a.spill_cap + pos] = h;
            return;
        }
    }
    wc_global_add(a, h, 1);
}

__device__ __forceinline__ void wc_local_add(uint64_t *sk, uint32_t *sc, uint32_t *scnt,
                                             const WcArgs &a, uint64_t h)
{
    if (h != 0) {
        uint32_t s = (uint32_t)h & (kWcSlots - 1);
        for (uint32_t p = 0; p < kWcProbes; ++p) {
            const uint64_t k = sk[s];
            if (k == h) {
                atomicAdd(&sc[s], 1u);
                return;
            }
            if (k == 0) {
                const uint64_t old =
                    atomicCAS((unsigned long long *)&sk[s], 0ull, (unsigned long long)h);
                if (old == 0 || old == h) {
                    atomicAdd(&sc[s], 1u);
                    return;
                }
            }
            s = (s + 1) & (kWcSlots - 1);
        }
    }
    wc_spill(scnt, a, h);
}

// 16 bytes of text at byte `pos` (a thread's span), bytes at or past n read
// as spaces, so no word starts or continues there.
__device__ __forceinline__ uint4 wc_span(const uint8_t *text, uint64_t n, uint64_t pos,
                                         bool vec)
{
    if (vec && pos + 16 <= n)
        return *reinterpret_cast<const uint4 *>(text + pos);
    uint32_t w[4] = {0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u};
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (pos + k < n) {
            const uint32_t sh = 8 * (k & 3);
            w[k >> 2] = (w[k >> 2] & ~(0xFFu << sh)) | ((uint32_t)text[pos + k] << sh);
        }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Bit i of the result is set when byte i of w (little-endian) is whitespace
// (wc_space), for the four bytes at once: with each byte's top bit forced to
// 1, the per-byte subtractions below cannot borrow across bytes, so the top
// bit of each byte of (w | 0x80..) - c tells whether its low 7 bits are >= c;
// bytes of 0x80 and above are never whitespace.
__device__ __forceinline__ uint32_t space_bits4(uint32_t w)
{
    const uint32_t top = 0x80808080u;
    const uint32_t up = w | top;
    const uint32_t ge09 = (up - 0x09090909u) & top;
    const uint32_t ge0e = (up - 0x0E0E0E0Eu) & top;
    const uint32_t ne20 = (((w ^ 0x20202020u) & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) & top;
    const uint32_t ws = ((ge09 & ~ge0e) | (~ne20 & top)) & ~w & top;
    return ((ws >> 7) & 1u) | ((ws >> 14) & 2u) | ((ws >> 21) & 4u) | ((ws >> 28) & 8u);
}

// Block barrier for LDS traffic only: waits for this wave's LDS operations,
// not for its global loads in flight (the next chunk's prefetch).
__device__ __forceinline__ void lds_barrier()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0); vmcnt, expcnt untouched
    __builtin_amdgcn_s_barrier();
    __asm__ __volatile__("" ::: "memory");
}

// The scan.  Per staged chunk: each thread marks the whitespace bytes of its
// 16-byte span in a bitmap (one 16-bit word per span, chunk and look-ahead)
// and the word starts in its span; a wave prefix sum places the starts in a
// per-wave list; then each lane takes whole words from the list, reads the
// word's length off the bitmap, hashes its bytes from the staged chunk and
// counts the key in the block's LDS table.  A word that runs past the
// look-ahead continues from the text in global memory, one byte at a time.
// The scan front end shared by counting and locating: the block's chunks of
// the text are staged in LDS, each wave lists its words' starts and hashes
// one word per lane; word(h, off) is called with the word's key and the byte
// offset of its first byte.  Returns the number of words this thread listed.
template <class Word>
__device__ __forceinline__ uint64_t wc_scan(const uint8_t *text, uint64_t n, Word word)
{
    constexpr uint32_t kLookSpans = kWcLook / 16;
    constexpr uint32_t kSpans = kBlock + kLookSpans;
    __shared__ uint4 st4[kSpans + 1];               // (+ 16 bytes read past the end)
    __shared__ uint32_t sepm[kSpans];               // whitespace bits of each span
    __shared__ uint16_t starts16[kWaves][64 * 8];   // a 16-byte span holds <= 8 word starts
    __shared__ uint32_t sh_prev;
    const uint8_t *st = reinterpret_cast<const uint8_t *>(st4);
    if (threadIdx.x == 0)
        st4[kSpans] = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
    const bool vec = ((uintptr_t)text & 15u) == 0;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    uint16_t *wl = starts16[wave];
    const uint64_t nchunks = (n + kWcChunk - 1) / kWcChunk;
    constexpr uint64_t kBasis = 14695981039346656037ull;
    // this thread's span of the first chunk, its look-ahead span and (thread
    // 0) the byte before the chunk, loaded ahead of use
    uint64_t c = blockIdx.x;
    uint4 cur = wc_span(text, n, c * kWcChunk + 16 * tid, vec);
    uint4 look = make_uint4(0, 0, 0, 0);
    if (tid < kLookSpans)
        look = wc_span(text, n, c * kWcChunk + kWcChunk + 16 * tid, vec);
    uint32_t prevb = (tid == 0 && c > 0 && c < nchunks) ? text[c * kWcChunk - 1] : 0x20u;
    uint64_t words = 0;
    for (; c < nchunks; c += gridDim.x) {
        const uint64_t c0 = c * kWcChunk;
        lds_barrier(); // the previous chunk's words are done with the staging
        const uint4 mine = cur;
        st4[tid] = mine;
        const uint32_t sep = space_bits4(mine.x) | (space_bits4(mine.y) << 4) |
                             (space_bits4(mine.z) << 8) | (space_bits4(mine.w) << 12);
        sepm[tid] = sep;
        if (tid < kLookSpans) {
            st4[kBlock + tid] = look;
            sepm[kBlock + tid] = space_bits4(look.x) | (space_bits4(look.y) << 4) |
                                 (space_bits4(look.z) << 8) | (space_bits4(look.w) << 12);
        }
        if (tid == 0)
            sh_prev = prevb;
        const uint64_t cn = c + gridDim.x;
        if (cn < nchunks) { // prefetch the block's next chunk
            cur = wc_span(text, n, cn * kWcChunk + 16 * tid, vec);
            if (tid < kLookSpans)
                look = wc_span(text, n, cn * kWcChunk + kWcChunk + 16 * tid, vec);
            if (tid == 0)
                prevb = text[cn * kWcChunk - 1];
        }
        lds_barrier(); // staged
        const uint32_t prev = tid ? st[16 * tid - 1] : sh_prev;
        uint32_t starts = ~sep & ((sep << 1) | (uint32_t)wc_space(prev)) & 0xFFFFu;
        const uint32_t mycount = __builtin_popcount(starts);
        // exclusive prefix sum of the word counts over the wave's lanes
        uint32_t incl = mycount;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o);
            if (lane >= (uint32_t)o)
                incl += v;
        }
        const uint32_t total = __shfl(incl, 63);
        uint32_t slot = incl - mycount;
        while (starts) {
            const uint32_t b = __builtin_ctz(starts);
            wl[slot++] = (uint16_t)(16 * tid + b);
            starts &= starts - 1;
        }
        words += mycount;
        // the wave's words: one per lane at a time
        for (uint32_t i = lane; i < total; i += 64) {
            const uint32_t s0 = wl[i];
            // length: the distance to the next whitespace bit at or after s0
            uint32_t span = s0 >> 4;
            uint32_t m = sepm[span] >> (s0 & 15u);
            uint32_t len = 0;
            bool ends = m != 0;
            if (ends) {
                len = __builtin_ctz(m);
            } else {
                len = 16u - (s0 & 15u);
                for (++span; span < kSpans; ++span) {
                    m = sepm[span];
                    if (m) {
                        len += __builtin_ctz(m);
                        ends = true;
                        break;
                    }
                    len += 16u;
                }
            }
            // the staged bytes of the word, four at a time
            uint64_t h = kBasis;
            for (uint32_t k = 0; k < len; k += 4) {
                const uint32_t b0 = st[s0 + k], b1 = st[s0 + k + 1];
                const uint32_t b2 = st[s0 + k + 2], b3 = st[s0 + k + 3];
                h = fnv_step(h, b0);
                if (k + 1 < len)
                    h = fnv_step(h, b1);
                if (k + 2 < len)
                    h = fnv_step(h, b2);
                if (k + 3 < len)
                    h = fnv_step(h, b3);
            }
            if (!ends) {
                // past the look-ahead: the rest from the text
                for (uint64_t j = c0 + s0 + len; j < n; ++j) {
                    const uint32_t byte = text[j];
                    if (wc_space(byte))
                        break;
                    h = fnv_step(h, byte);
                }
            }
            word(h, c0 + s0);
        }
    }
    return words;
}

__global__ __launch_bounds__(kBlock) void k_wordcount(WcArgs a)
{
    __shared__ uint64_t sk[kWcSlots];
    __shared__ uint32_t sc[kWcSlots];
    __shared__ uint32_t scnt[1u << kWcPartBits];    // spill appends per partition
    for (uint32_t i = threadIdx.x; i < kWcSlots; i += kBlock) {
        sk[i] = 0;
        sc[i] = 0;
    }
    for (uint32_t i = threadIdx.x; i < (1u << kWcPartBits); i += kBlock)
        scnt[i] = 0;
    uint64_t words = wc_scan(a.text, a.n, [&](uint64_t h, uint64_t) {
        wc_local_add(sk, sc, scnt, a, h);
    });
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    __syncthreads();
    for (uint32_t i = tid; i < kWcSlots; i += kBlock)
        if (sk[i])
            wc_global_add(a, sk[i], sc[i]);
    if (a.spill_cap != 0)
        for (uint32_t p = tid; p < (1u << kWcPartBits); p += kBlock)
            a.spill_cnt[((uint64_t)blockIdx.x << kWcPartBits) | p] = min(scnt[p], a.spill_cap);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        words += __shfl_xor(words, o);
    if (lane == 0 && words)
        atomicAdd((unsigned long long *)&a.ctl[0], (unsigned long long)words);
}

// ---- WordCount's words: the first occurrence of each key --------------------
// A lookup table from key to the key's index in the caller's array (open
// addressing at load <= 1/2, key 0 = empty; the key 0 itself is kept in
// ctl[0] as index + 1), then one pass of the scan front end in which every
// word whose key is in the table lowers that key's offset to its own with an
// atomic minimum.  A word reads the key's current offset first and skips the
// atomic when that is already lower, so after a key's first few words its
// later ones cost one load.
__global__ __launch_bounds__(kBlock) void k_wl_build(WlArgs l)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= l.nkeys)
        return;
    l.offsets[i] = ~0ull;
    const uint64_t h = l.keys[i];
    if (h == 0) {
        if (atomicCAS((unsigned long long *)&l.ctl[0], 0ull, (unsigned long long)(i + 1)) != 0)
            atomicOr((unsigned long long *)&l.ctl[1], 1ull); // the key 0 twice
        return;
    }
    uint64_t s = h & l.mask;
    for (uint64_t probe = 0; probe <= l.mask; ++probe) {
        const uint64_t old =
            atomicCAS((unsigned long long *)&l.tkeys[s], 0ull, (unsigned long long)h);
        if (old == 0) {
            l.tidx[s] = (uint32_t)i;
            return;
        }
        if (old == h) {
            atomicOr((unsigned long long *)&l.ctl[1], 1ull); // a key twice
            return;
        }
        s = (s + 1) & l.mask;
    }
}

__global__ __launch_bounds__(kBlock) void k_wl_scan(WlArgs l)
{
    (void)wc_scan(l.text, l.n, [&](uint64_t h, uint64_t off) {
        uint64_t idx = ~0ull;
        if (h == 0) {
            const uint64_t z = l.ctl[0];
            if (z)
                idx = z - 1;
        } else {
            // the table is at most half full, so a probe run ends at an
            // empty slot
            for (uint64_t s = h & l.mask;; s = (s + 1) & l.mask) {
                const uint64_t k = l.tkeys[s];
                if (k == h) {
                    idx = l.tidx[s];
                    break;
                }
                if (k == 0)
                    break;
            }
        }
        if (idx != ~0ull && l.offsets[idx] > off)
            atomicMin((unsigned long long *)&l.offsets[idx], (unsigned long long)off);
    });
}

// Merge of the spill regions: block b counts partition b / per_part's keys
// from the regions of the scan blocks congruent to b modulo per_part in an
// LDS table, then adds each distinct key it holds to the global table once.
// Each thread walks one region at a time (a few hundred bytes), sixteen
// keys in flight, so the block has many regions' loads outstanding at once.
// Keys that find no LDS slot go to the table directly.
constexpr uint32_t kWcMergeSlots = 2048;
constexpr uint32_t kWcMergeProbes = 8;

__device__ __forceinline__ void wc_merge_add(uint64_t *mk, uint32_t *mc, const WcArgs &a,
                                             uint64_t h)
{
    uint32_t s = (uint32_t)h & (kWcMergeSlots - 1);
    for (uint32_t q = 0; q < kWcMergeProbes; ++q) {
        const uint64_t key = mk[s];
        if (key == h) {
            atomicAdd(&mc[s], 1u);
            return;
        }
        if (key == 0) {
            const uint64_t old =
                atomicCAS((unsigned long long *)&mk[s], 0ull, (unsigned long long)h);
            if (old == 0 || old == h) {
                atomicAdd(&mc[s], 1u);
                return;
            }
        }
        s = (s + 1) & (kWcMergeSlots - 1);
    }
    wc_global_add(a, h, 1);
}

__global__ __launch_bounds__(kBlock) void k_wc_merge(WcArgs a, uint32_t scan_grid,
                                                    uint32_t per_part)
{
    __shared__ uint64_t mk[kWcMergeSlots];
    __shared__ uint32_t mc[kWcMergeSlots];
    for (uint32_t i = threadIdx.x; i < kWcMergeSlots; i += kBlock) {
        mk[i] = 0;
        mc[i] = 0;
    }
    __syncthreads();
    const uint32_t p = blockIdx.x / per_part, k = blockIdx.x % per_part;
    constexpr uint32_t kInFlight = 16;
    for (uint64_t b = k + (uint64_t)per_part * threadIdx.x; b < scan_grid;
         b += (uint64_t)per_part * kBlock) {
        const uint64_t r = (b << kWcPartBits) | p;
        const uint32_t cnt = a.spill_cnt[r];
        const uint64_t *src = a.spill + r * a.spill_cap;
        for (uint32_t i = 0; i < cnt; i += kInFlight) {
            uint64_t h[kInFlight];
#pragma unroll
            for (uint32_t u = 0; u < kInFlight; ++u)
                h[u] = i + u < cnt ? src[i + u] : 0;
            // one copy of the insert, the keys rotated through h[0] (sixteen
            // inlined copies of it left the compiler spilling hundreds of
            // scalar registers)
#pragma unroll 1
            for (uint32_t u = 0; u < kInFlight; ++u) {
                const uint64_t key = h[0];
#pragma unroll
                for (uint32_t v = 0; v + 1 < kInFlight; ++v)
                    h[v] = h[v + 1];
                if (key) // spilled keys are never 0
                    wc_merge_add(mk, mc, a, key);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kWcMergeSlots; i += kBlock)
        if (mk[i])
            wc_global_add(a, mk[i], mc[i]);
}

// Compaction of the global table into the caller's key/count arrays
// (unordered); ctl[3] counts the distinct keys, also those past `cap`.  Each
// block owns a contiguous range of slots: it counts its keys, reserves room
// with one atomic add (a counter bumped once per key would serialise on
// that one address), then writes its keys in slot order at its offset.
__global__ __launch_bounds__(kBlock) void k_wc_compact(WcArgs a, uint64_t *out_keys,
                                                      uint64_t *out_counts, uint64_t cap)
{
    __shared__ uint32_t sh_wave[kWaves];
    __shared__ uint64_t sh_base;
    const uint64_t slots = a.mask + 1;
    const uint64_t per = (slots + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = min(slots, (uint64_t)blockIdx.x * per);
    const uint64_t hi = min(slots, lo + per);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    // pass 1: this block's key count
    uint32_t mine = 0;
    for (uint64_t s = lo + threadIdx.x; s < hi; s += kBlock)
        mine += a.keys[s] != 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        mine += __shfl_xor(mine, o);
    if (lane == 0)
        sh_wave[wave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0;
        for (int w = 0; w < kWaves; ++w)
            total += sh_wave[w];
        sh_base = total ? atomicAdd((unsigned long long *)&a.ctl[3], (unsigned long long)total)
                        : 0;
    }
    __syncthreads();
    // pass 2: keys in slot order, kBlock slots at a time, placed by a block
    // prefix sum of the occupied slots
    uint64_t base = sh_base;
    __syncthreads();
    for (uint64_t s0 = lo; s0 < hi; s0 += kBlock) {
        const uint64_t s = s0 + threadIdx.x;
        const uint64_t k = s < hi ? a.keys[s] : 0;
        const uint64_t ballot = __ballot(k != 0);
        const uint32_t before = __popcll(ballot & ((1ull << lane) - 1));
        if (lane == 0)
            sh_wave[wave] = __popcll(ballot);
        __syncthreads();
        uint32_t off = 0, total = 0;
        for (int w = 0; w < kWaves; ++w) {
            off += w < (int)wave ? sh_wave[w] : 0;
            total += sh_wave[w];
        }
        if (k != 0) {
            const uint64_t pos = base + off + before;
            if (pos < cap) {
                out_keys[pos] = k;
                out_counts[pos] = a.counts[s];
            }
        }
        base += total;
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.ctl[1]) {
        const uint64_t pos = atomicAdd((unsigned long long *)&a.ctl[3], 1ull);
        if (pos < cap) {
            out_keys[pos] = 0;
            out_counts[pos] = a.ctl[1];
        }
    }
}

// Synthetic data for the autotuner: a cheap hash pattern in [-1, 1).
__global__ __launch_bounds__(kBlock) void k_fill_pattern(float *p, uint64_t n,
                                                         uint32_t salt)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ salt;
        h ^= h >> 15;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        p[i] = (float)((int32_t)(h >> 8) - (1 << 23)) * (1.0f / 8388608.0f);
    }
}

// ---- resident serving executor -------------------------------------------
// Block 0 is the dispatcher: it polls the host ring's tail word (system
// scope), copies each new descriptor into the device table, writes the task's
// tiles into the tile map and publishes the new tile count.  Every other block
// is a worker.  A worker takes one tile ticket at a time with an atomic add
// (one round trip, no retries), then polls the published-tile word with
// exponential backoff until its ticket is published, and runs the tile
// exactly as the batch executor does; a task's last tile writes its result to
// host memory and then its completion word.  Every wait is bounded: the
// dispatcher leaves on the host's stop word, or after idle_ticks without new
// work, setting the stop bit of the published-tile word (and the abort bit
// when the host asked to abort).  A worker leaves only on the abort bit, or
// when the stop bit is set and its ticket is unpublished: a claimed ticket is
// never given up while the dispatcher lives, however long the wait for its
// tile (under a light load the highest claims wait for hundreds of tasks).
// The stop bit is or-ed into the final published count, so a worker that sees
// it also sees every tile that will ever be published in this launch.
// Tickets are issued in order and a worker never leaves holding a published
// ticket, so every published tile runs before the grid drains.  A ticket left
// unpublished at exit is discarded by the next launch's prologue, which
// restarts the tickets at the published count.  A dispatcher that stops
// polling would leave the workers waiting; the host's watchdog covers that
// case (it aborts the launch).

static_assert(offsetof(TaskDev, ntiles) == 96, "word 24 of a descriptor");
static_assert(offsetof(TaskDev, tile_first) == 120, "words 30-31 of a descriptor");

// Descriptors copied per round of the dispatcher: one per 32-thread group, so
// a burst of arrivals costs one host-memory round trip per 8 tasks.
constexpr uint32_t kServeBatch = kBlock / 32;

__device__ __forceinline__ void serve_dispatch(const ServeArgs &a)
{
    __shared__ uint64_t sh_tail, sh_stop;
    __shared__ uint32_t sh_nt[kServeBatch], sh_first_lo[kServeBatch], sh_first_hi[kServeBatch];
    uint64_t taken = uni64(ld_agent(&a.dev->taken));
    uint64_t last = wall_clock64();
    for (;;) {
        if (threadIdx.x == 0) {
            sh_tail = __hip_atomic_load(&a.host->tail, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_SYSTEM);
            sh_stop = __hip_atomic_load(&a.host->stop, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
        const uint64_t tail = uni64(sh_tail);
        const uint32_t stop = uni((uint32_t)sh_stop);
        __syncthreads();
        if (stop) {
            if (threadIdx.x == 0 && stop >= 2)
                __hip_atomic_fetch_or(&a.dev->tiles_pub, kServeAbortBit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        if (tail > taken) {
            uint64_t pub = 0;
            // Descriptors taken .. tail-1, kServeBatch at a time: group g of
            // 32 threads copies descriptor s0 + g (one 32-bit word per
            // thread) from the host ring to the device table and writes its
            // tile-map entries.  The tile ranges of different descriptors are
            // disjoint (the host assigned them), so the groups work apart.
            const uint32_t g = threadIdx.x >> 5, l = threadIdx.x & 31u;
            for (uint64_t s0 = taken; s0 < tail; s0 += kServeBatch) {
                const uint64_t s = s0 + g;
                const uint32_t slot = (uint32_t)(s & (a.cap - 1));
                uint32_t nt = 0;
                uint64_t first = 0;
                if (s < tail) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                    uint32_t *src = reinterpret_cast<uint32_t *>(
                                        const_cast<TaskDev *>(a.ring + slot)) + l;
                    uint32_t *dst = reinterpret_cast<uint32_t *>(a.table + slot) + l;
                    const uint32_t w = __hip_atomic_load(src, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(dst, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (l == 24)
                        sh_nt[g] = w;
                    if (l == 30)
                        sh_first_lo[g] = w;
                    if (l == 31)
                        sh_first_hi[g] = w;
                }
                __syncthreads();
                if (s < tail) {
                    nt = sh_nt[g];
                    first = ((uint64_t)sh_first_hi[g] << 32) | sh_first_lo[g];
                    for (uint32_t k = l; k < nt; k += 32)
                        __hip_atomic_store(a.tilemap + ((first + k) & (a.tile_cap - 1)), slot,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                // the last descriptor of the round ends the published range
                const uint32_t last = (uint32_t)min((uint64_t)kServeBatch, tail - s0) - 1;
                pub = (((uint64_t)uni(sh_first_hi[last]) << 32) | uni(sh_first_lo[last])) +
                      uni(sh_nt[last]);
                __syncthreads();
            }
            // table and tile-map entries were written with agent-scope atomic
            // stores; once they are complete the new tile count is published
            own_stores_complete();
            __syncthreads();
            if (threadIdx.x == 0) {
                st_agent(&a.dev->taken, tail);
                own_stores_complete();
                st_agent(&a.dev->tiles_pub, pub);
            }
            taken = tail;
            last = wall_clock64();
            continue;
        }
        if (wall_clock64() - last > a.idle_ticks)
            break;
        __builtin_amdgcn_s_sleep(16);
    }
    if (threadIdx.x == 0)
        __hip_atomic_fetch_or(&a.dev->tiles_pub, kServeStopBit, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void serve_work(const ServeArgs &a)
{
    __shared__ uint64_t sh_tile;
    __shared__ TaskDev sh_task;
    constexpr uint64_t kNone = ~0ull;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint64_t c = __hip_atomic_fetch_add(&a.dev->claim, 1ull, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            uint64_t got = kNone;
            uint32_t backoff = 1;
            for (;;) {
                const uint64_t w = ld_agent(&a.dev->tiles_pub);
                if (w & kServeAbortBit)
                    break;
                if (c < (w & kServeCountMask)) {
                    got = c;
                    break;
                }
                if (w & kServeStopBit)
                    break;
                // s_sleep takes an immediate: a few fixed steps of backoff
                if (backoff == 1)
                    __builtin_amdgcn_s_sleep(1);
                else if (backoff == 2)
                    __builtin_amdgcn_s_sleep(4);
                else
                    __builtin_amdgcn_s_sleep(16);
                backoff = backoff < 3 ? backoff + 1 : 3;
            }
            sh_tile = got;
        }
        __syncthreads();
        const uint64_t t = uni64(sh_tile);
        if (t == kNone)
            break;
        // Acquire before touching the task: the descriptor, and the task's
        // inputs, which the caller may have rewritten since this resident
        // kernel last read that memory (its L2 is not invalidated between
        // tasks the way it is between kernel launches).
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x < 32) {
            const uint32_t slot = __hip_atomic_load(a.tilemap + (t & (a.tile_cap - 1)),
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t *src = reinterpret_cast<uint32_t *>(a.table + slot) + threadIdx.x;
            reinterpret_cast<uint32_t *>(&sh_task)[threadIdx.x] =
                __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const uint32_t j = uni((uint32_t)(t - sh_task.tile_first));
        run_tile(&sh_task, j, a.out);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_serve(ServeArgs a)
{
    if (blockIdx.x == 0)
        serve_dispatch(a);
    else
        serve_work(a);
}

// Launch prologue: clear the stop bit and restart the tickets at the
// published count (no worker of the previous launch is alive to hold one).
__global__ void k_serve_prologue(ServeDev *d)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint64_t pub = d->tiles_pub & kServeCountMask;
        d->tiles_pub = pub;
        d->claim = pub;
    }
}

int hip_status(hipError_t e)
{
    return e == hipSuccess ? SPARKCL_OK : SPARKCL_EHIP;
}

} // namespace

int launch_task(const TaskDev *dtask, uint32_t ntiles, uint32_t grid,
                const LaunchOut &out, void *stream, uint32_t block)
{
    if (block != 256 && block != 512 && block != 1024)
        return SPARKCL_EINVAL;
    if (ntiles == 0 || grid == 0)
        return SPARKCL_EINVAL;
    grid = grid < ntiles ? grid : ntiles;
    hipLaunchKernelGGL(k_task, dim3(grid), dim3(block), 0, (hipStream_t)stream,
                       dtask, out);
    return hip_status(hipGetLastError());
}

int launch_chain(const TaskDev *dtasks, const TileRef *tiles, uint32_t ntiles,
                 const ChainDev *chain, uint32_t grid, const LaunchOut &out, uint32_t unroll,
                 void *stream)
{
    if (ntiles == 0 || grid == 0 || !chain || (unroll != 4 && unroll != 8))
        return SPARKCL_EINVAL;
    if (unroll == 8)
        hipLaunchKernelGGL(k_chain<8>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                           dtasks, tiles, ntiles, chain, out);
    else
        hipLaunchKernelGGL(k_chain<4>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                           dtasks, tiles, ntiles, chain, out);
    return hip_status(hipGetLastError());
}

int launch_batch(const TaskDev *dtasks, const TileRef *tiles, uint32_t ntiles,
                 uint32_t grid, const LaunchOut &out, void *stream, uint32_t block,
                 bool mc_only)
{
    if (ntiles == 0 || grid == 0 || (block != 256 && block != 512 && block != 1024))
        return SPARKCL_EINVAL;
    if (mc_only)
        hipLaunchKernelGGL(k_batch_mc, dim3(grid), dim3(block), 0, (hipStream_t)stream,
                           dtasks, tiles, ntiles, out);
    else
        hipLaunchKernelGGL(k_batch, dim3(grid), dim3(block), 0, (hipStream_t)stream,
                           dtasks, tiles, ntiles, out);
    return hip_status(hipGetLastError());
}

int launch_map(const TaskDev *dtask, uint64_t n, uint32_t variant, uint32_t grid,
               void *stream)
{
    if (grid == 0)
        return SPARKCL_EINVAL;
    hipLaunchKernelGGL(k_map, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       dtask, n, variant);
    return hip_status(hipGetLastError());
}

int launch_wordcount(const WcArgs &a, uint32_t grid, void *stream)
{
    if (grid == 0 || !a.keys || !a.counts || !a.ctl || ((a.mask + 1) & a.mask) ||
        (a.spill_cap != 0 && (!a.spill || !a.spill_cnt)))
        return SPARKCL_EINVAL;
    hipLaunchKernelGGL(k_wordcount, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, a);
    return hip_status(hipGetLastError());
}

int launch_wc_merge(const WcArgs &a, uint32_t scan_grid, uint32_t per_part, void *stream)
{
    if (a.spill_cap == 0 || scan_grid == 0 || per_part == 0)
        return SPARKCL_EINVAL;
    const uint32_t grid = per_part << kWcPartBits;
    hipLaunchKernelGGL(k_wc_merge, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, a,
                       scan_grid, per_part);
    return hip_status(hipGetLastError());
}

int launch_wc_compact(const WcArgs &a, uint64_t *keys, uint64_t *counts, uint64_t cap,
                      uint32_t grid, void *stream)
{
    if (grid == 0)
        return SPARKCL_EINVAL;
    hipLaunchKernelGGL(k_wc_compact, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, a,
                       keys, counts, cap);
    return hip_status(hipGetLastError());
}

int launch_wordcount_locate(const WlArgs &l, uint32_t scan_grid, void *stream)
{
    if (scan_grid == 0 || !l.offsets || !l.tkeys || !l.tidx || !l.ctl ||
        ((l.mask + 1) & l.mask) || (l.nkeys && !l.keys) || l.nkeys > 0xFFFFFFFFull ||
        2 * l.nkeys > l.mask + 1)
        return SPARKCL_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (l.nkeys) {
        const uint64_t bgrid = (l.nkeys + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_wl_build, dim3((uint32_t)bgrid), dim3(kBlock), 0, s, l);
        const int rc = hip_status(hipGetLastError());
        if (rc != SPARKCL_OK)
            return rc;
    }
    if (l.n)
        hipLaunchKernelGGL(k_wl_scan, dim3(scan_grid), dim3(kBlock), 0, s, l);
    return hip_status(hipGetLastError());
}

int wordcount_blocks_per_cu(int *out)
{
    return hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        out, reinterpret_cast<const void *>(k_wordcount), kBlock, 0));
}

int launch_tree(const TreeArgs &a, uint32_t combiner, bool vec4, void *stream)
{
    if (a.len == 0 || a.count == 0 || a.chunk == 0)
        return SPARKCL_EINVAL;
    const uint32_t nchunks = (a.count + a.chunk - 1) / a.chunk;
    if (nchunks > 1 && (a.chunk & (a.chunk - 1)))
        return SPARKCL_EINVAL;
    if (a.chunk > (1u << (kTreeSlots - 1)) || nchunks > 65535)
        return SPARKCL_EINVAL;
    if (vec4 && (a.len & 3u))
        return SPARKCL_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (a.cpt != 1) {
        if (!vec4 || (a.cpt != 2 && a.cpt != 4) || a.chunk > kTreeWideChunk ||
            (combiner != SPARKCL_VADD && combiner != SPARKCL_VMAX) ||
            (a.threads != (uint32_t)kBlock && !(a.threads == kTreeWideBig && a.cpt == 4)))
            return SPARKCL_EINVAL;
        const uint64_t per_block = (uint64_t)a.threads * a.cpt;
        const uint64_t cb = ((a.len >> 2) + per_block - 1) / per_block;
        if (cb > 0x7fffffffull)
            return SPARKCL_EINVAL;
        const dim3 grid((uint32_t)cb, nchunks);
        const dim3 block(a.threads);
        if (combiner == SPARKCL_VADD) {
            if (a.threads == kTreeWideBig)
                hipLaunchKernelGGL((k_tree_wide<SPARKCL_VADD, 4, kTreeWideBig>), grid, block, 0, s, a);
            else if (a.cpt == 4)
                hipLaunchKernelGGL((k_tree_wide<SPARKCL_VADD, 4, kBlock>), grid, block, 0, s, a);
            else
                hipLaunchKernelGGL((k_tree_wide<SPARKCL_VADD, 2, kBlock>), grid, block, 0, s, a);
        } else {
            if (a.threads == kTreeWideBig)
                hipLaunchKernelGGL((k_tree_wide<SPARKCL_VMAX, 4, kTreeWideBig>), grid, block, 0, s, a);
            else if (a.cpt == 4)
                hipLaunchKernelGGL((k_tree_wide<SPARKCL_VMAX, 4, kBlock>), grid, block, 0, s, a);
            else
                hipLaunchKernelGGL((k_tree_wide<SPARKCL_VMAX, 2, kBlock>), grid, block, 0, s, a);
        }
        return hip_status(hipGetLastError());
    }
    const uint32_t V = vec4 ? 4 : 1;
    const uint64_t colblocks = (a.len + (uint64_t)kBlock * V - 1) / ((uint64_t)kBlock * V);
    if (colblocks > 0x7fffffffull)
        return SPARKCL_EINVAL;
    const dim3 grid((uint32_t)colblocks, nchunks);
    if (combiner == SPARKCL_VADD) {
        if (vec4)
            hipLaunchKernelGGL((k_tree<4, SPARKCL_VADD>), grid, dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_tree<1, SPARKCL_VADD>), grid, dim3(kBlock), 0, s, a);
    } else if (combiner == SPARKCL_VMAX) {
        if (vec4)
            hipLaunchKernelGGL((k_tree<4, SPARKCL_VMAX>), grid, dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_tree<1, SPARKCL_VMAX>), grid, dim3(kBlock), 0, s, a);
    } else {
        return SPARKCL_EINVAL;
    }
    return hip_status(hipGetLastError());
}

int launch_zero(void *p, uint64_t bytes, void *stream)
{
    if (bytes % 4 != 0 || ((uintptr_t)p & 3u))
        return SPARKCL_EINVAL;
    const uint64_t words = bytes / 4;
    if (words == 0)
        return SPARKCL_OK;
    uint64_t grid = (words + kBlock - 1) / kBlock;
    if (grid > 4096)
        grid = 4096;
    hipLaunchKernelGGL(k_zero, dim3((uint32_t)grid), dim3(kBlock), 0,
                       (hipStream_t)stream, (uint32_t *)p, words);
    return hip_status(hipGetLastError());
}

int launch_fill_pattern(float *p, uint64_t n, uint32_t salt, void *stream)
{
    if (n == 0)
        return SPARKCL_OK;
    uint64_t grid = (n + kBlock - 1) / kBlock;
    if (grid > 8192)
        grid = 8192;
    hipLaunchKernelGGL(k_fill_pattern, dim3((uint32_t)grid), dim3(kBlock), 0,
                       (hipStream_t)stream, p, n, salt);
    return hip_status(hipGetLastError());
}

int launch_serve(const ServeArgs &a, uint32_t workers, void *stream)
{
    if (workers == 0 || a.cap == 0 || (a.cap & (a.cap - 1)) || a.tile_cap == 0 ||
        (a.tile_cap & (a.tile_cap - 1)))
        return SPARKCL_EINVAL;
    hipLaunchKernelGGL(k_serve_prologue, dim3(1), dim3(64), 0, (hipStream_t)stream, a.dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_status(e);
    hipLaunchKernelGGL(k_serve, dim3(workers + 1), dim3(kBlock), 0, (hipStream_t)stream, a);
    return hip_status(hipGetLastError());
}

int batch_blocks_per_cu(int *out)
{
    return hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        out, reinterpret_cast<const void *>(k_batch), kBlock, 0));
}

int batch_mc_blocks_per_cu(int *out)
{
    return hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        out, reinterpret_cast<const void *>(k_batch_mc), kBlock, 0));
}

int chain_blocks_per_cu(int *out)
{
    return hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        out, reinterpret_cast<const void *>(k_chain<4>), kBlock, 0));
}

} // namespace sparkcl
