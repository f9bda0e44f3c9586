// Autotuner: picks, by the lowest median HIP-event time on synthetic device
// data, first each registry kernel's persistent-executor blocks per CU
// jointly with its tile for large (2^22-element) partitions, then its block
// size (256, 512, 1024 threads) and, for the streaming kernels, its float4
// loads in flight per thread (2, 4, 8), then the tile size per execution
// mode, kernel and log2(n) bucket, then the tiles, occupancy and block size
// for batches of many small tasks of mixed kernels (tuned on a batch drawn
// from a distribution of its own, not the benchmark's).  The result is a tuning table
// that is written to a JSON cache keyed by the device's gfx arch, so a given
// machine always decomposes a task the same way (results stay run-to-run
// identical).  The paper leaves optimisation open (sec. 6); this is ours.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "runtime.h"
#include "serve.h"

using namespace sparkcl;

namespace {

// Synthetic input per array (1 GiB): batches stream from HBM, not from the
// 256 MB last-level cache.
constexpr uint64_t kPoolElems = 1ull << 28;
constexpr int kWarm = 3, kReps = 9;

// Elements per timed batch: 2^28 for the streaming kernels (1 GiB per input
// array; the tiles per block, not the launch, dominate, as in a large RDD)
// and 2^30 samples (about 1 ms) for the Monte-Carlo kernel, enough tiles for
// the Monte-Carlo-only executor's high occupancies to show.
uint64_t work_elems(uint32_t kid)
{
    return kid == SPARKCL_MC_PI ? (1ull << 30) : (1ull << 28);
}

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Bench {
    sparkcl_ctx *ctx;
    float *x = nullptr, *y = nullptr;
    hipStream_t s = nullptr;
};

// Median time (ms) of one reduce of `tasks` in `mode` under the context's
// current tuning table.
int time_reduce(Bench &b, int mode, const std::vector<sparkcl_task> &tasks, float *ms)
{
    Plan *p = nullptr;
    int rc = get_plan(b.ctx, 0, mode, tasks.data(), (uint32_t)tasks.size(), nullptr,
                      nullptr, b.s, &p);
    if (rc != SPARKCL_OK)
        return rc;
    std::vector<float> t;
    for (int r = 0; r < kWarm + kReps; ++r) {
        if ((rc = enqueue(b.ctx, p, b.s, true)) != SPARKCL_OK)
            return rc;
        SPARKCL_HIP(hipEventSynchronize(b.ctx->ev1));
        float v = 0;
        SPARKCL_HIP(hipEventElapsedTime(&v, b.ctx->ev0, b.ctx->ev1));
        if (r >= kWarm)
            t.push_back(v);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return SPARKCL_OK;
}

sparkcl_task make_task(const Bench &b, uint32_t kid, uint64_t n, uint64_t i)
{
    sparkcl_task t;
    std::memset(&t, 0, sizeof(t));
    t.kernel_id = kid;
    t.n = n;
    const uint64_t off = (i * n) % (kPoolElems - n + 1);
    if (kid == SPARKCL_MC_PI) {
        t.reduce_ops = SPARKCL_COUNT;
        t.partition_id = (uint32_t)i;
    } else {
        t.reduce_ops = SPARKCL_SUM | SPARKCL_MAX;
        t.in0 = b.x + off;
        t.in1 = kid == SPARKCL_FMUL ? b.y + off : nullptr;
        t.degree = 2;
        t.coef[0] = 3.0f;
        t.coef[1] = -1.25f;
        t.coef[2] = 0.5f;
        t.c = 0.1f;
    }
    return t;
}

// Many tasks of mixed kernels, shaped like an uneven RDD but not like any
// one benchmark: 3000 tasks with log-normal sizes (median 2^15, log-sd ln 5,
// clipped to [2^9, 2^22]) and kernel ids 2 : 2 : 1 (POLY : FMUL : MC_PI).
std::vector<sparkcl_task> make_mixed(const Bench &b)
{
    std::vector<sparkcl_task> v;
    uint64_t off = 0;
    for (uint64_t i = 0; i < 3000; ++i) {
        const uint64_t h1 = mix64(0x7a11e000 + 2 * i), h2 = mix64(0x7a11e001 + 2 * i);
        const double u1 = ((double)(h1 >> 11) + 0.5) * 0x1p-53;
        const double u2 = (double)(h2 >> 11) * 0x1p-53;
        const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
        const double e = std::log(32768.0) + std::log(5.0) * z;
        const uint64_t n = (uint64_t)std::min(4194304.0, std::max(512.0, std::rint(std::exp(e))));
        const uint32_t r5 = (uint32_t)((mix64(h1 ^ h2) >> 32) % 5);
        const uint32_t kid = r5 < 2 ? SPARKCL_POLY : r5 < 4 ? SPARKCL_FMUL : SPARKCL_MC_PI;
        sparkcl_task t = make_task(b, kid, n, 0);
        if (kid != SPARKCL_MC_PI) {
            if (off + n > kPoolElems)
                off = 0;
            t.in0 = b.x + off;
            t.in1 = kid == SPARKCL_FMUL ? b.y + off : nullptr;
            off += n;
        }
        v.push_back(t);
    }
    return v;
}

std::vector<sparkcl_task> make_tasks(const Bench &b, uint32_t kid, uint64_t n, int mode,
                                     uint64_t work = 0)
{
    const uint64_t count =
        mode == SPARKCL_BATCHED ? std::max<uint64_t>(1, (work ? work : work_elems(kid)) / n) : 1;
    std::vector<sparkcl_task> v;
    for (uint64_t i = 0; i < std::min<uint64_t>(count, 4096); ++i)
        v.push_back(make_task(b, kid, n, i));
    return v;
}

} // namespace

extern "C" int sparkcl_autotune(sparkcl_ctx *ctx, uint32_t lo_log2, uint32_t hi_log2,
                                const char *path)
{
    if (!ctx)
        return fail(SPARKCL_EINVAL, "null context");
    if (lo_log2 > hi_log2 || hi_log2 > 24)
        return fail(SPARKCL_EINVAL, "bucket range must satisfy lo <= hi <= 24");
    SPARKCL_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->mu);

    Bench b;
    b.ctx = ctx;
    const uint64_t xoff = ctx->arena.alloc(kPoolElems * 4);
    const uint64_t yoff = ctx->arena.alloc(kPoolElems * 4);
    auto cleanup = [&]() {
        drop_plans(ctx);
        if (xoff != Arena::kFail)
            ctx->arena.release(xoff);
        if (yoff != Arena::kFail)
            ctx->arena.release(yoff);
        if (b.s)
            (void)hipStreamDestroy(b.s);
    };
    if (xoff == Arena::kFail || yoff == Arena::kFail) {
        cleanup();
        return fail(SPARKCL_ENOMEM, "autotune needs 2 GiB of free arena");
    }
    b.x = static_cast<float *>(ctx->dev(xoff));
    b.y = static_cast<float *>(ctx->dev(yoff));
    int rc;
    if (hipStreamCreateWithFlags(&b.s, hipStreamNonBlocking) != hipSuccess ||
        (rc = launch_fill_pattern(b.x, kPoolElems, 0x1234u, b.s)) != SPARKCL_OK ||
        (rc = launch_fill_pattern(b.y, kPoolElems, 0xBEEFu, b.s)) != SPARKCL_OK ||
        hipStreamSynchronize(b.s) != hipSuccess) {
        cleanup();
        return fail(SPARKCL_EHIP, "autotune setup failed");
    }

    sparkcl_tuning best = ctx->tuning;
    const bool verbose = std::getenv("SPARKCL_AUTOTUNE_LOG") != nullptr;
    // Times `tasks` under tuning `t`; false (with rc set) on failure.
    auto measure = [&](const sparkcl_tuning &t, int mode,
                       const std::vector<sparkcl_task> &tasks, float *ms) -> bool {
        drop_plans(ctx);
        ctx->tuning = t;
        rc = time_reduce(b, mode, tasks, ms);
        return rc == SPARKCL_OK;
    };
    // A batched candidate the plan would not take (its blocks would get
    // fewer than two tiles each, and the plan then cuts the batch with the
    // per-launch table) is not measured, so no entry records a tile size
    // that never ran.
    auto batched_takes = [&](const sparkcl_tuning &t, uint32_t kid,
                             const std::vector<sparkcl_task> &tasks, uint32_t T) {
        uint64_t tiles = 0;
        for (const sparkcl_task &x : tasks)
            tiles += std::max<uint64_t>(1, (x.n + T - 1) / T);
        const sparkcl_tuning keep = ctx->tuning;
        ctx->tuning = t;
        const uint64_t grid = exec_grid(ctx, 1u << (kid - 1), tiles, tasks.size());
        ctx->tuning = keep;
        return tiles >= 2 * grid;
    };
    auto abort_with = [&](int code) {
        ctx->tune_shared_mc = false;
        ctx->tuning = best;
        cleanup();
        return code;
    };
    const uint32_t occ = (uint32_t)ctx->occ_batch;

    // 1. Executor blocks per CU and the large-partition tile, jointly, per
    //    kernel, on a 2^28-element batch of 2^22-element partitions (tiles and
    //    occupancy trade against each other: large tiles want more blocks).
    //    Ties (within 2%) go to fewer blocks and smaller tiles.
    constexpr uint32_t kRefLog2 = 22;
    for (uint32_t kid = SPARKCL_POLY; kid <= SPARKCL_MC_PI; ++kid) {
        // Monte-Carlo tasks are first timed on the shared executor, where
        // only mixed batches use blocks_per_cu[MC_PI], at the Monte-Carlo
        // share such a batch carries (2^27 samples; the 4096-task uneven
        // batch holds 2.1e8); the instance that runs them alone is tuned
        // after (1c) on the full 2^30
        const std::vector<sparkcl_task> tasks =
            kid == SPARKCL_MC_PI ? make_tasks(b, kid, 1ull << kRefLog2, SPARKCL_BATCHED, 1ull << 27)
                                 : make_tasks(b, kid, 1ull << kRefLog2, SPARKCL_BATCHED);
        ctx->tune_shared_mc = kid == SPARKCL_MC_PI;
        const uint32_t kocc = exec_occupancy(ctx, 1u << (kid - 1));
        float best_ms = 1e30f;
        uint32_t best_bpc = 1, best_tile = best.tile[TM_BATCHED][kid - 1][kRefLog2];
        for (uint32_t bpc = 1; bpc <= kocc; ++bpc)
            for (uint32_t tl = 14; tl <= 20; ++tl) {
                sparkcl_tuning t = best;
                t.blocks_per_cu[kid - 1] = bpc;
                t.tile[TM_BATCHED][kid - 1][kRefLog2] = 1u << tl;
                if (!batched_takes(t, kid, tasks, 1u << tl))
                    continue;
                float ms = 0;
                if (!measure(t, SPARKCL_BATCHED, tasks, &ms))
                    return abort_with(rc);
                if (verbose)
                    std::fprintf(stderr, "joint kid %u bpc %u tile 2^%u: %.1f us\n", kid, bpc,
                                 tl, ms * 1e3f);
                if (ms < best_ms * 0.98f) {
                    best_ms = ms;
                    best_bpc = bpc;
                    best_tile = 1u << tl;
                }
            }
        best.blocks_per_cu[kid - 1] = best_bpc;
        best.tile[TM_BATCHED][kid - 1][kRefLog2] = best_tile;

        // 1b. Blocks per CU, block size and loads in flight jointly at that
        //     tile, against the step-1 choice (256 threads, 4 loads), which a
        //     candidate must beat by 2%; then the tile again at the chosen
        //     shape.  Blocks per CU count 256-thread blocks (a 512-thread
        //     block takes two), so a bigger block needs as many of them.
        //     On MI355X the joint search matters: POLY streamed 2^22-element
        //     partitions fastest at 1 block per CU with 8 loads in flight, a
        //     point that neither one-dimensional search visits.
        {
            float shape_ms = best_ms;
            const sparkcl_tuning base = best;
            for (uint32_t blk : {256u, 512u, 1024u})
                for (uint32_t bpc = blk / 256; bpc <= kocc; ++bpc)
                    for (uint32_t u : {4u, 2u, 8u}) {
                        if (kid == SPARKCL_MC_PI && u != 4)
                            continue; // no streaming loop
                        if (blk == 256 && u == 4 && bpc == best_bpc)
                            continue; // the step-1 choice
                        sparkcl_tuning t = base;
                        t.blocks_per_cu[kid - 1] = bpc;
                        t.block[kid - 1] = blk;
                        t.unroll[kid - 1] = u;
                        if (!batched_takes(t, kid, tasks, best_tile))
                            continue;
                        float ms = 0;
                        if (!measure(t, SPARKCL_BATCHED, tasks, &ms))
                            return abort_with(rc);
                        if (verbose)
                            std::fprintf(stderr,
                                         "shape kid %u block %u bpc %u unroll %u: %.1f us\n",
                                         kid, blk, bpc, u, ms * 1e3f);
                        if (ms < shape_ms * 0.98f) {
                            shape_ms = ms;
                            best.blocks_per_cu[kid - 1] = bpc;
                            best.block[kid - 1] = blk;
                            best.unroll[kid - 1] = u;
                        }
                    }
            for (uint32_t tl = 14; tl <= 20; ++tl) {
                sparkcl_tuning t = best;
                t.tile[TM_BATCHED][kid - 1][kRefLog2] = 1u << tl;
                if ((1u << tl) == best_tile || !batched_takes(t, kid, tasks, 1u << tl))
                    continue;
                float ms = 0;
                if (!measure(t, SPARKCL_BATCHED, tasks, &ms))
                    return abort_with(rc);
                if (verbose)
                    std::fprintf(stderr, "retile kid %u tile 2^%u: %.1f us\n", kid, tl,
                                 ms * 1e3f);
                if (ms < shape_ms * 0.98f) {
                    shape_ms = ms;
                    best.tile[TM_BATCHED][kid - 1][kRefLog2] = 1u << tl;
                }
            }
        }

        // 1c. Monte-Carlo tasks alone: the blocks per CU of the executor
        //     instance that holds only the Philox body, at the tile above.
        ctx->tune_shared_mc = false;
        if (kid == SPARKCL_MC_PI) {
            const std::vector<sparkcl_task> alone =
                make_tasks(b, kid, 1ull << kRefLog2, SPARKCL_BATCHED);
            const uint32_t mocc = exec_occupancy(ctx, 1u << (kid - 1));
            const uint32_t T = best.tile[TM_BATCHED][kid - 1][kRefLog2];
            float mc_ms = 1e30f;
            for (uint32_t bpc = 1; bpc <= mocc; ++bpc) {
                sparkcl_tuning t = best;
                t.blocks_per_cu_mc_only = bpc;
                if (!batched_takes(t, kid, alone, T))
                    continue;
                float ms = 0;
                if (!measure(t, SPARKCL_BATCHED, alone, &ms))
                    return abort_with(rc);
                if (verbose)
                    std::fprintf(stderr, "mc alone bpc %u: %.1f us\n", bpc, ms * 1e3f);
                if (ms < mc_ms * 0.98f) {
                    mc_ms = ms;
                    best.blocks_per_cu_mc_only = bpc;
                }
            }
        }
    }

    // 2. Tile size per (mode, kernel, log2-size bucket) at those occupancies.
    const int modes[2] = {SPARKCL_PER_LAUNCH, SPARKCL_BATCHED};
    for (int mode : modes) {
        const int tm = mode == SPARKCL_BATCHED ? TM_BATCHED : TM_PER_LAUNCH;
        for (uint32_t kid = SPARKCL_POLY; kid <= SPARKCL_MC_PI; ++kid) {
            for (uint32_t bk = lo_log2; bk <= hi_log2; ++bk) {
                if (tm == TM_BATCHED && bk == kRefLog2)
                    continue; // tuned jointly above
                const uint64_t n = 1ull << bk;
                const std::vector<sparkcl_task> tasks = make_tasks(b, kid, n, mode);
                float best_ms = 1e30f;
                uint32_t best_tile = best.tile[tm][kid - 1][bk];
                for (uint32_t tl = kMinTileLog2; tl <= kMaxTileLog2; ++tl) {
                    const uint32_t T = 1u << tl;
                    if (T > std::max<uint64_t>(n, 1u << kMinTileLog2))
                        break;
                    if (n / T > (1u << 20))
                        continue;
                    sparkcl_tuning t = best;
                    t.tile[tm][kid - 1][bk] = T;
                    if (tm == TM_BATCHED && !batched_takes(t, kid, tasks, T))
                        continue;
                    float ms = 0;
                    if (!measure(t, mode, tasks, &ms))
                        return abort_with(rc);
                    if (verbose)
                        std::fprintf(stderr, "tile mode %d kid %u n 2^%u T 2^%u: %.1f us\n",
                                     mode, kid, bk, tl, ms * 1e3f);
                    if (ms < best_ms * 0.98f) { // prefer the earlier (smaller) on ties
                        best_ms = ms;
                        best_tile = T;
                    }
                }
                best.tile[tm][kid - 1][bk] = best_tile;
            }
        }
    }

    // 3-5. The mixed batch (many tasks of spread sizes and mixed kernels,
    //    drawn from a distribution of its own): its occupancy, which a batch
    //    that mixes kernels takes alone; the work shares (tiles per CU) that
    //    its streaming input bytes (both streaming kernels, whose tiles run
    //    side by side in HBM), then its Monte-Carlo samples, are cut into,
    //    against the per-bucket table (0); the occupancy again at those
    //    shares; then the executor's block size.  Explicit mixed-batch tile
    //    sizes are left unset: a size tuned on one batch does not carry over
    //    to a batch of another total, a share does.
    {
        const std::vector<sparkcl_task> tasks = make_mixed(b);
        best.tile_many[0] = best.tile_many[1] = best.tile_many[2] = 0;
        auto tune_many_bpc = [&]() -> bool {
            float best_ms = 1e30f;
            uint32_t best_bpc = best.blocks_per_cu_many;
            for (uint32_t bpc = 1; bpc <= occ; ++bpc) {
                sparkcl_tuning t = best;
                t.blocks_per_cu_many = bpc;
                float ms = 0;
                if (!measure(t, SPARKCL_BATCHED, tasks, &ms))
                    return false;
                if (verbose)
                    std::fprintf(stderr, "many bpc %u: %.1f us\n", bpc, ms * 1e3f);
                if (ms < best_ms * 0.98f) {
                    best_ms = ms;
                    best_bpc = bpc;
                }
            }
            best.blocks_per_cu_many = best_bpc;
            return true;
        };
        if (!tune_many_bpc())
            return abort_with(rc);
        for (int group = 0; group < 2; ++group) {
            float best_ms = 1e30f;
            uint32_t best_q = 0;
            for (uint32_t q : {0u, 4u, 8u, 12u, 16u, 24u, 32u, 48u, 64u, 128u}) { // 0: the table
                sparkcl_tuning t = best;
                t.many_tiles_per_cu[group] = q;
                float ms = 0;
                if (!measure(t, SPARKCL_BATCHED, tasks, &ms))
                    return abort_with(rc);
                if (verbose)
                    std::fprintf(stderr, "mixed %s tiles per CU %u: %.1f us\n",
                                 group == 0 ? "streaming" : "mc_pi", q, ms * 1e3f);
                if (ms < best_ms * 0.98f) {
                    best_ms = ms;
                    best_q = q;
                }
            }
            best.many_tiles_per_cu[group] = best_q;
        }
        if (!tune_many_bpc())
            return abort_with(rc);

        float shape_ms = 1e30f;
        for (uint32_t blk : {256u, 512u, 1024u}) {
            sparkcl_tuning t = best;
            t.block_many = blk;
            float ms = 0;
            if (!measure(t, SPARKCL_BATCHED, tasks, &ms))
                return abort_with(rc);
            if (verbose)
                std::fprintf(stderr, "many block %u: %.1f us\n", blk, ms * 1e3f);
            if (ms < shape_ms * 0.98f) {
                shape_ms = ms;
                best.block_many = blk;
            }
        }
    }

    ctx->tuning = best;
    if (ctx->server)
        ctx->server->set_tuning(best);
    cleanup();
    if (path) {
        std::string err;
        if (!tuning_save_file(path, ctx->arch, best, &err))
            return fail(SPARKCL_EINVAL, err);
    }
    return SPARKCL_OK;
}
