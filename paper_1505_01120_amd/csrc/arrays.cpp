// Array-valued ReduceCL (sec. 3.1.3; Fig 3; SparkCLVectorAdd, sec. 3.2.2): the
// RDD's elements are float arrays of one length, folded by a two-input
// combiner along a fixed pairwise tree.  Plans (leaf tables, passes and their
// intermediate rows) are cached in the context like the reduce plans.
#include <algorithm>
#include <cstring>
#include <string>

#include "runtime.h"

using namespace sparkcl;

namespace {

constexpr uint32_t kTreeMaxK = 1u << 24;
constexpr uint32_t kTreeMaxChunk = 4096; // leaves per chunk the kernel's counter holds
constexpr uint32_t kTreeMaxChunks = 65535;

uint32_t pow2_floor(uint64_t v)
{
    uint32_t p = 1;
    while ((uint64_t)p * 2 <= v && p < (1u << 31))
        p *= 2;
    return p;
}

// Array reduces are keyed by kind (2: pointer table, 3: rows of one buffer),
// combiner, shape, output and the leaves (the table, or base and stride).
uint64_t tree_hash(int kind, uint32_t combiner, const float *const *arrays,
                   const float *base, uint64_t stride, uint32_t k, uint64_t len,
                   const float *out)
{
    uint64_t h = 0xCBF29CE484222325ull;
    h = fnv1a(h, &kind, sizeof(kind));
    h = fnv1a(h, &combiner, sizeof(combiner));
    h = fnv1a(h, &k, sizeof(k));
    h = fnv1a(h, &len, sizeof(len));
    h = fnv1a(h, &out, sizeof(out));
    h = fnv1a(h, &base, sizeof(base));
    h = fnv1a(h, &stride, sizeof(stride));
    return arrays ? fnv1a(h, arrays, sizeof(const float *) * k) : h;
}

bool tree_plan_matches(const Plan *p, int kind, uint64_t h, uint32_t combiner,
                       const float *const *arrays, const float *base, uint64_t stride,
                       uint32_t k, uint64_t len, const float *out)
{
    if (p->kind != kind || p->hash != h || p->combiner != combiner || p->len != len ||
        p->user_out != out || p->nleaves != k || p->leaf_base != base ||
        p->leaf_stride != stride)
        return false;
    return !arrays ||
           std::memcmp(p->leaves.data(), arrays, sizeof(const float *) * k) == 0;
}

// Splits the reduction into passes: each pass folds chunks of `chunk` leaves
// (a power of two unless it is the last pass), with enough chunks that the
// grid fills the GPU when the arrays are short, and writes one row per
// chunk; the next pass folds those rows.
int build_tree_plan(sparkcl_ctx *ctx, uint32_t combiner, const float *const *arrays,
                    const float *base, uint64_t stride, uint32_t k, uint64_t len,
                    float *out, hipStream_t stream, Plan **res)
{
    std::unique_ptr<Plan> p(new Plan);
    p->kind = arrays ? 2 : 3;
    p->combiner = combiner;
    p->len = len;
    p->user_out = out;
    p->nleaves = k;
    p->leaf_base = base;
    p->leaf_stride = stride;
    // float4 columns whenever the length is a multiple of 4: leaves and out
    // need only their 4-byte alignment (a 16-byte access at a 4-byte-aligned
    // address is one dwordx4 instruction)
    const bool vec4 = (len & 3u) == 0;
    if (arrays) {
        p->leaves.assign(arrays, arrays + k);
        for (uint32_t i = 0; i < k; ++i) {
            if (!arrays[i])
                return fail(SPARKCL_EINVAL, "array " + std::to_string(i) + " is NULL");
            if ((uintptr_t)arrays[i] & 3u)
                return fail(SPARKCL_EINVAL, "arrays must be 4-byte aligned");
        }
    }
    p->vec4 = vec4;
    const uint64_t V = vec4 ? 4 : 1;
    const uint64_t colblocks = (len + kBlock * V - 1) / (kBlock * V);
    const uint64_t target = 4ull * (uint64_t)ctx->cus; // blocks that fill the GPU

    std::vector<uint32_t> rows; // output rows of each pass
    uint32_t count = k;
    for (;;) {
        uint32_t chunk = 0, cpt = 1, threads = kBlock;
        // float4 columns: the wide kernel (leaf pairs, 2 or 4 columns per
        // thread, chunks of up to 64 leaves) when its grid still fills half
        // the GPU's block slots and at most one more pass follows (many
        // short columns fold better in the deeper chunks of the 8-leaf
        // kernel: 65536 rows of 4096 floats took 189 us through 64-leaf
        // chunks and four passes, 181 us in three); the most columns per
        // thread first, in blocks of kTreeWideBig threads when those alone
        // give every CU two blocks (64 arrays of 2^22 floats: 163 us against
        // 170 us in 256-thread blocks)
        if (vec4) {
            const uint32_t ch = std::min<uint32_t>(count, kTreeWideChunk);
            const uint64_t nch = (count + (uint64_t)ch - 1) / ch;
            const uint64_t cb_big = (len / 4 + kTreeWideBig * 4ull - 1) / (kTreeWideBig * 4ull);
            if (nch <= kTreeWideChunk && cb_big * nch >= 2ull * (uint64_t)ctx->cus) {
                cpt = 4;
                threads = kTreeWideBig;
                chunk = ch;
            }
            for (uint32_t c : {4u, 2u}) {
                if (cpt > 1)
                    break;
                const uint64_t cb = (len / 4 + (uint64_t)kBlock * c - 1) / ((uint64_t)kBlock * c);
                if (nch <= kTreeWideChunk && cb * nch >= target / 2) {
                    cpt = c;
                    chunk = ch;
                    break;
                }
            }
        }
        // One pass when the columns alone fill the GPU (then long per-thread
        // chains are hidden by other waves) or the chain is short; else fold
        // chunks so the grid of columns x chunks fills the GPU.
        if (cpt > 1) {
            // chosen above
        } else if (count <= kTreeMaxChunk && (colblocks >= target || count <= 64)) {
            chunk = count; // final pass
        } else {
            chunk = pow2_floor(std::max<uint64_t>(1, (uint64_t)count * colblocks / target));
            chunk = std::max<uint32_t>(chunk, 8);
            chunk = std::min<uint32_t>(chunk, kTreeMaxChunk);
            while ((count + (uint64_t)chunk - 1) / chunk > kTreeMaxChunks)
                chunk *= 2;
            if (chunk >= count)
                chunk = count;
        }
        const uint32_t nchunks = (uint32_t)((count + (uint64_t)chunk - 1) / chunk);
        TreeArgs a{};
        a.len = len;
        a.count = count;
        a.chunk = chunk;
        a.cpt = cpt;
        a.threads = threads;
        p->passes.push_back(a);
        rows.push_back(nchunks);
        if (nchunks == 1)
            break;
        count = nchunks;
    }

    // scratch: rows of pass 0 in buffer 0, of pass 1 in buffer 1, then alternate
    float *scratch[2] = {nullptr, nullptr};
    for (size_t i = 0; i + 1 < p->passes.size() && i < 2; ++i) {
        const uint64_t bytes = (uint64_t)rows[i] * len * 4;
        void *q = nullptr;
        int rc = arena_alloc(ctx, p.get(), std::max<uint64_t>(bytes, 256), &q);
        if (rc != SPARKCL_OK) {
            Plan *raw = p.release();
            free_plan(ctx, raw);
            return rc;
        }
        scratch[i] = static_cast<float *>(q);
    }
    void *dptrs = nullptr;
    if (arrays) {
        int rc = arena_alloc(ctx, p.get(), sizeof(const float *) * k, &dptrs);
        if (rc != SPARKCL_OK) {
            Plan *raw = p.release();
            free_plan(ctx, raw);
            return rc;
        }
    }
    for (size_t i = 0; i < p->passes.size(); ++i) {
        TreeArgs &a = p->passes[i];
        if (i == 0) {
            a.ptrs = static_cast<const float *const *>(dptrs);
            a.base = base;
            a.stride = stride;
        } else {
            a.base = scratch[(i - 1) % 2];
            a.stride = len;
        }
        a.out = (i + 1 == p->passes.size()) ? out : scratch[i % 2];
    }
    if (arrays) {
        hipError_t e = hipMemcpyAsync(dptrs, p->leaves.data(), sizeof(const float *) * k,
                                      hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            Plan *raw = p.release();
            free_plan(ctx, raw);
            return fail_hip(e, "upload of the array table");
        }
    }
    p->hash = tree_hash(p->kind, combiner, arrays, base, stride, k, len, out);
    *res = p.release();
    return SPARKCL_OK;
}

} // namespace

namespace {

int reduce_tree(sparkcl_ctx *ctx, uint32_t combiner, const float *const *arrays,
                const float *base, uint64_t stride, uint32_t k, uint64_t len, float *out,
                void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (combiner != SPARKCL_VADD && combiner != SPARKCL_VMAX)
        return fail(SPARKCL_EINVAL, "combiner " + std::to_string(combiner) +
                                        " is not SPARKCL_VADD or SPARKCL_VMAX");
    if (k == 0 || (!arrays && !base))
        return fail(SPARKCL_EINVAL, "an array reduce needs at least one array");
    if (k > kTreeMaxK)
        return fail(SPARKCL_ETOOBIG, "more than 2^24 arrays");
    if (len > kMaxN)
        return fail(SPARKCL_ETOOBIG, "arrays longer than 2^40 elements");
    if (!arrays && (((uintptr_t)base & 3u) || (k > 1 && stride < len)))
        return fail(SPARKCL_EINVAL, "rows must be 4-byte aligned and row_stride >= len");
    if (len == 0)
        return SPARKCL_OK;
    if (!out)
        return fail(SPARKCL_EINVAL, "out is NULL");
    if ((uintptr_t)out & 3u)
        return fail(SPARKCL_EINVAL, "out must be 4-byte aligned");
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int kind = arrays ? 2 : 3;
    const uint64_t h = tree_hash(kind, combiner, arrays, base, stride, k, len, out);
    Plan *p = nullptr;
    for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it)
        if (tree_plan_matches(*it, kind, h, combiner, arrays, base, stride, k, len, out)) {
            p = *it;
            ctx->plans.splice(ctx->plans.begin(), ctx->plans, it);
            break;
        }
    if (!p) {
        if (capturing(s))
            return fail(SPARKCL_EINVAL, "no cached plan for this call on a stream under capture: "
                                        "make the same call once before capturing");
        while (ctx->plans.size() >= kMaxPlans)
            evict_one(ctx);
        if ((rc = build_tree_plan(ctx, combiner, arrays, base, stride, k, len, out, s, &p)) !=
            SPARKCL_OK)
            return rc;
        ctx->plans.push_front(p);
    }
    for (const TreeArgs &a : p->passes)
        if ((rc = launch_tree(a, combiner, p->vec4, s)) != SPARKCL_OK)
            return fail(rc, "array reduce launch failed");
    return SPARKCL_OK;
}

} // namespace

extern "C" {

int sparkcl_reduce_arrays(sparkcl_ctx *ctx, uint32_t combiner, const float *const *arrays,
                          uint32_t k, uint64_t len, float *out, void *stream)
{
    if (k && !arrays)
        return fail(SPARKCL_EINVAL, "arrays is NULL");
    return reduce_tree(ctx, combiner, arrays, nullptr, 0, k, len, out, stream);
}

int sparkcl_reduce_rows(sparkcl_ctx *ctx, uint32_t combiner, const float *base,
                        uint64_t row_stride, uint32_t k, uint64_t len, float *out,
                        void *stream)
{
    if (k && !base)
        return fail(SPARKCL_EINVAL, "base is NULL");
    return reduce_tree(ctx, combiner, nullptr, base, row_stride, k, len, out, stream);
}

} // extern "C"
