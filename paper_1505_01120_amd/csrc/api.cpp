// C ABI of the SparkCL map -> reduce hot path (include/sparkcl.h).
//
// Execution model: a call's tasks are validated, decomposed into tiles by the
// tuning table, and uploaded once into arena memory as a Plan (device task
// table, tile queue, partial slots, sync words, results).  Plans are cached by
// the content of the call, so a repeated batch skips validation and upload
// and is one kernel dispatch of the persistent executor (the kernel leaves
// its queue and tickets at zero, so nothing is cleared between launches).
// This is
// the paper's point that a kernel should be instantiated once per worker and
// cached (sec. 3.1.1.2), and that enough data must be gathered per offload
// (sec. 3, issue 2).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "runtime.h"
#include "serve.h"

using namespace sparkcl;

namespace sparkcl {

namespace {
thread_local std::string t_last_error;
constexpr uint32_t kStagingSlots = 3; // host-input partitions in flight
} // namespace

int fail(int code, const std::string &msg)
{
    t_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(SPARKCL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t host_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int check_task(const sparkcl_task &t, uint32_t *variant)
{
    if (t.kernel_id < SPARKCL_POLY || t.kernel_id > SPARKCL_MC_PI)
        return fail(SPARKCL_ENOKERNEL, "kernel id " + std::to_string(t.kernel_id) +
                                           " is not in the registry");
    if (t.n > kMaxN)
        return fail(SPARKCL_ETOOBIG, "partition of " + std::to_string(t.n) +
                                         " elements exceeds 2^40");
    if (t.flags & ~SPARKCL_TASK_HOST_INPUT)
        return fail(SPARKCL_EINVAL, "unknown task flags");
    if (t.flags & SPARKCL_TASK_HOST_INPUT) {
        if (t.kernel_id == SPARKCL_MC_PI)
            return fail(SPARKCL_EINVAL, "MC_PI has no input arrays to stream from the host");
        if (t.out)
            return fail(SPARKCL_EINVAL, "host-input tasks take out == NULL");
    }
    if (t.kernel_id == SPARKCL_MC_PI) {
        if (t.reduce_ops != SPARKCL_COUNT)
            return fail(SPARKCL_EINVAL, "MC_PI takes reduce_ops == SPARKCL_COUNT");
        *variant = V_MC;
        return SPARKCL_OK;
    }
    if (t.reduce_ops == 0 || (t.reduce_ops & ~(SPARKCL_SUM | SPARKCL_MAX)))
        return fail(SPARKCL_EINVAL, "POLY/FMUL take a non-empty subset of SUM|MAX");
    if (t.n > 0 && !t.in0)
        return fail(SPARKCL_EINVAL, "in0 is NULL with n > 0");
    if (t.kernel_id == SPARKCL_FMUL && t.n > 0 && !t.in1)
        return fail(SPARKCL_EINVAL, "FMUL needs in1");
    if (((uintptr_t)t.in0 | (uintptr_t)t.in1 | (uintptr_t)t.out) & 3u)
        return fail(SPARKCL_EINVAL, "arrays must be 4-byte aligned");
    if (t.kernel_id == SPARKCL_POLY) {
        if (t.degree > 7)
            return fail(SPARKCL_EINVAL, "POLY degree above 7");
        *variant = (t.out ? V_POLYW : V_POLY) + t.degree;
    } else {
        *variant = t.out ? V_FMULW : V_FMUL;
    }
    return SPARKCL_OK;
}

uint64_t input_bytes(uint32_t kernel_id)
{
    return kernel_id == SPARKCL_FMUL ? 8ull : 4ull;
}

uint64_t offload_cost(const sparkcl_task &t)
{
    return t.n * input_bytes(t.kernel_id);
}

bool declined(const sparkcl_ctx *ctx, const sparkcl_task &t)
{
    return ctx->config.offload_min_bytes && offload_cost(t) < ctx->config.offload_min_bytes;
}


// FNV-style hash over 8-byte words (byte tail folded in), for plan lookup.
uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        std::memcpy(&w, b + i, 8);
        h = (h ^ w) * 0x100000001B3ull;
    }
    for (; i < n; ++i)
        h = (h ^ b[i]) * 0x100000001B3ull;
    return h;
}

uint64_t plan_hash(int kind, int mode, const sparkcl_task *tasks, uint32_t ntasks,
                   const void *ures, const void *utot)
{
    uint64_t h = 0xCBF29CE484222325ull;
    h = fnv1a(h, &kind, sizeof(kind));
    h = fnv1a(h, &mode, sizeof(mode));
    h = fnv1a(h, &ntasks, sizeof(ntasks));
    h = fnv1a(h, &ures, sizeof(ures));
    h = fnv1a(h, &utot, sizeof(utot));
    return fnv1a(h, tasks, sizeof(sparkcl_task) * ntasks);
}

void free_plan(sparkcl_ctx *ctx, Plan *p)
{
    for (hipEvent_t e : p->ev_copied)
        if (e)
            (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_copied2)
        if (e)
            (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_done)
        if (e)
            (void)hipEventDestroy(e);
    if (p->ev_start)
        (void)hipEventDestroy(p->ev_start);
    for (hipGraphExec_t &x : p->gexec)
        if (x)
            (void)hipGraphExecDestroy(x);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    for (uint64_t off : p->blocks)
        ctx->arena.release(off);
    delete p;
}

// Evicts the least recently used plan; waits for the device first so no
// in-flight launch still uses its memory.  False if nothing is left.
bool evict_one(sparkcl_ctx *ctx)
{
    if (ctx->plans.empty())
        return false;
    (void)hipDeviceSynchronize();
    Plan *p = ctx->plans.back();
    ctx->plans.pop_back();
    free_plan(ctx, p);
    return true;
}

int arena_alloc(sparkcl_ctx *ctx, Plan *p, uint64_t bytes, void **out)
{
    for (;;) {
        uint64_t off = ctx->arena.alloc(bytes);
        if (off != Arena::kFail) {
            p->blocks.push_back(off);
            *out = ctx->dev(off);
            return SPARKCL_OK;
        }
        if (!evict_one(ctx))
            return fail(SPARKCL_ENOMEM, "arena exhausted: need " + std::to_string(bytes) +
                                            " bytes, largest free block " +
                                            std::to_string(ctx->arena.largest_free()));
    }
}

} // namespace sparkcl

uint32_t sparkcl::exec_block(const sparkcl_ctx *ctx, uint32_t kid_mask)
{
    uint32_t b = ctx->tuning.block_many;
    for (uint32_t k = 0; k < 3; ++k)
        if (kid_mask == (1u << k))
            b = ctx->tuning.block[k];
    return b ? b : (uint32_t)kBlock;
}

uint32_t sparkcl::kernel_unroll(const sparkcl_tuning &t, uint32_t kid)
{
    const uint32_t u = kid >= SPARKCL_POLY && kid <= SPARKCL_MC_PI ? t.unroll[kid - 1] : 0;
    return u ? u : (uint32_t)kUnroll;
}

uint32_t sparkcl::exec_occupancy(const sparkcl_ctx *ctx, uint32_t kid_mask)
{
    return (uint32_t)(mc_instance(ctx, kid_mask) ? ctx->occ_mc : ctx->occ_batch);
}

bool sparkcl::mc_instance(const sparkcl_ctx *ctx, uint32_t kid_mask)
{
    return kid_mask == (1u << (SPARKCL_MC_PI - 1)) && !ctx->tune_shared_mc;
}

uint32_t sparkcl::exec_grid(const sparkcl_ctx *ctx, uint32_t kid_mask, uint64_t ntiles,
                            uint64_t ntasks, uint32_t block)
{
    // a batch of Monte-Carlo tasks alone runs the executor's MC instance,
    // which fits more blocks per CU
    const uint32_t occ = exec_occupancy(ctx, kid_mask);
    uint32_t per_cu = 0;
    if (ctx->config.exec_blocks_per_cu) {
        per_cu = ctx->config.exec_blocks_per_cu;
    } else if (kid_mask == (1u << (SPARKCL_MC_PI - 1)) && !ctx->tune_shared_mc) {
        // Monte-Carlo tasks alone: the executor instance of their own
        per_cu = ctx->tuning.blocks_per_cu_mc_only ? ctx->tuning.blocks_per_cu_mc_only : occ;
    } else {
        // the largest tuned value among the kernels in the batch: a
        // compute-bound kernel needs waves to hide instruction latency, a
        // streaming one does best with a few deep streams per CU
        for (uint32_t k = 0; k < 3; ++k)
            if (kid_mask & (1u << k)) {
                const uint32_t v = ctx->tuning.blocks_per_cu[k];
                per_cu = std::max(per_cu, v ? v : occ);
            }
        if (per_cu == 0)
            per_cu = occ;
        // many small tasks: per-tile latency (queue, descriptor, ticket,
        // final combine) has to be hidden by more blocks per CU
        if (ntasks && ntiles < 4 * ntasks) {
            const uint32_t v = ctx->tuning.blocks_per_cu_many;
            per_cu = std::max(per_cu, v ? v : occ);
        }
    }
    // per_cu counts 256-thread blocks (waves per SIMD); larger blocks take
    // their share of them
    const uint32_t waves = std::max(1u, std::min(per_cu, occ));
    if (block == 0)
        block = exec_block(ctx, kid_mask);
    return std::max(1u, waves * (uint32_t)kBlock / block) * (uint32_t)ctx->cus;
}

sparkcl::Cut sparkcl::plan_cut(const sparkcl_ctx *ctx, int mode, const sparkcl_task *tasks,
                                uint32_t ntasks, bool host_in, uint32_t per_cu)
{
    // Tile table: the batched one, unless the batch would then give the
    // executor's blocks fewer than two tiles each (a batch of one or a few
    // partitions, where the batched table's large tiles would leave most of
    // the GPU idle, or about one large tile per block, where the time is set
    // by how unevenly the blocks land on the CUs); such a batch is cut with
    // the per-launch table instead.  The choice is a function of the call,
    // so a repeated call is cut the same way.
    Cut c;
    c.tm = mode != SPARKCL_PER_LAUNCH && !host_in ? TM_BATCHED : TM_PER_LAUNCH;
    // A batch of many tasks of widely spread sizes takes the mixed-batch
    // tile sizes instead of the per-bucket table (tuned on batches of one
    // size): one tile size per kernel, so small tasks run whole and large
    // ones in mid-sized interleaved tiles.  On the 4096-task uneven batch one
    // 2^16 tile for the streaming kernels ran it in 515 us against 553 us
    // with the table.  The size is either given (tile_many) or derived from
    // the batch's own total work, cut into a tuned number of tiles per CU:
    // the share, not the size, is what carries over between batches.
    // Streaming work is counted in input bytes, so a POLY tile (4 bytes per
    // element) holds twice the elements of an FMUL tile (8): tiles of equal
    // bytes stream for equal times and carry equal shares of the per-tile
    // set-up (on the uneven batch, 2^16 POLY with 2^15 FMUL elements ran in
    // 461 us against 471 us with 2^16 for both).
    if (c.tm == TM_BATCHED && ntasks >= kMixedMinTasks) {
        uint32_t lo = SPARKCL_TUNE_BUCKETS, hi = 0;
        uint64_t total[2] = {0, 0}; // streaming input bytes, Monte-Carlo samples
        for (uint32_t i = 0; i < ntasks; ++i) {
            const uint32_t b = size_bucket(tasks[i].n);
            lo = std::min(lo, b);
            hi = std::max(hi, b);
            if (tasks[i].kernel_id == SPARKCL_MC_PI)
                total[1] += tasks[i].n;
            else if (tasks[i].kernel_id == SPARKCL_POLY || tasks[i].kernel_id == SPARKCL_FMUL)
                total[0] += tasks[i].n * input_bytes(tasks[i].kernel_id);
        }
        c.mixed = hi >= lo + kMixedMinSpan;
        for (uint32_t kid = SPARKCL_POLY; kid <= SPARKCL_MC_PI && c.mixed; ++kid) {
            const int k = kid == SPARKCL_MC_PI ? 1 : 0;
            const uint32_t q = ctx->tuning.many_tiles_per_cu[k];
            if (q == 0 || total[k] == 0)
                continue;
            const double per_elem = k == 1 ? 1.0 : (double)input_bytes(kid);
            const double want = (double)total[k] / ((double)ctx->cus * q) / per_elem;
            const double l2 = std::rint(std::log2(std::max(want, 1.0)));
            const int e = (int)std::min<double>(kMaxTileLog2, std::max<double>(kMinTileLog2, l2));
            c.share_tile[kid - 1] = 1u << e;
        }
    }
    if (c.tm == TM_BATCHED) {
        uint64_t tiles = 0;
        uint32_t mask = 0;
        for (uint32_t i = 0; i < ntasks; ++i) {
            if (tasks[i].kernel_id < SPARKCL_POLY || tasks[i].kernel_id > SPARKCL_MC_PI)
                continue; // rejected by check_task
            const uint32_t T = cut_tile(ctx, c, tasks[i]);
            tiles += std::max<uint64_t>(1, (tasks[i].n + T - 1) / T);
            mask |= 1u << (tasks[i].kernel_id - 1);
        }
        const uint64_t grid =
            per_cu ? per_cu * (uint32_t)ctx->cus : exec_grid(ctx, mask, tiles, ntasks);
        if (tiles < 2 * grid) {
            c.tm = TM_PER_LAUNCH;
            c.mixed = false;
            c.share_tile[0] = c.share_tile[1] = c.share_tile[2] = 0;
        }
    }
    return c;
}

uint32_t sparkcl::cut_tile(const sparkcl_ctx *ctx, const Cut &c, const sparkcl_task &t)
{
    if (c.tm == TM_BATCHED && c.mixed && t.kernel_id >= SPARKCL_POLY &&
        t.kernel_id <= SPARKCL_MC_PI) {
        if (ctx->tuning.tile_many[t.kernel_id - 1])
            return ctx->tuning.tile_many[t.kernel_id - 1];
        const uint32_t s = c.share_tile[t.kernel_id - 1];
        if (s)
            return s;
    }
    return tile_for(ctx->tuning, c.tm, t.kernel_id, t.n);
}

void sparkcl::fill_taskdev(const sparkcl_task &t, uint32_t variant, uint32_t tile,
                           uint32_t ntiles, uint32_t index, Partial *partials, uint32_t unroll,
                           TaskDev *d)
{
    std::memset(d, 0, sizeof(*d));
    d->kid = (uint16_t)t.kernel_id;
    d->unroll = (uint16_t)unroll;
    d->ops = t.reduce_ops;
    d->n = t.n;
    d->in0 = t.in0;
    d->in1 = t.in1;
    d->out = t.out;
    d->seed = t.seed;
    d->pid = t.partition_id;
    d->variant = variant;
    std::memcpy(d->coef, t.coef, sizeof(d->coef));
    d->c = t.c;
    d->tile_elems = tile;
    d->ntiles = ntiles;
    d->index = index;
    d->partials = partials;
}

void sparkcl::queue_tiles(const sparkcl_task *tasks, uint32_t ntasks, const TaskDev *dev,
                          uint32_t *order, uint32_t *mem, uint32_t *alu, TileRef *tiles)
{
    // Tile queue, longest tiles first (a longest-processing-time list
    // schedule: the batch then ends on short tiles instead of leaving a few
    // blocks streaming large tiles while the rest idle).  A tile's cost is
    // its element count times the kernel's cost per element (bytes streamed;
    // a Monte-Carlo sample counts like ~5 bytes of HBM time).  Ties keep task
    // order and each task's tiles together and in order, so the tiles of a
    // task still run side by side.  The order only changes when tiles run:
    // every partial and every combine order is fixed by the decomposition,
    // so results are unaffected.
    auto per_elem = [&](uint32_t i) -> uint64_t {
        const uint32_t kid = tasks[i].kernel_id;
        return kid == SPARKCL_POLY ? 4 : kid == SPARKCL_FMUL ? 8 : 5;
    };
    auto cost = [&](uint32_t i) -> uint64_t {
        return dev[i].variant == V_DECLINED
                   ? 0
                   : std::min<uint64_t>(dev[i].tile_elems, tasks[i].n) * per_elem(i);
    };
    for (uint32_t i = 0; i < ntasks; ++i)
        order[i] = i;
    // (an index tie-break makes the unstable in-place sort stable)
    std::sort(order, order + ntasks, [&](uint32_t a, uint32_t b) {
        const uint64_t ca = cost(a), cb = cost(b);
        return ca > cb || (ca == cb && a < b);
    });
    // Memory-bound (POLY, FMUL) and VALU-bound (MC_PI) tasks use different
    // units, so the two longest-first lists are merged to advance through the
    // same fraction of their work: at every point of the queue, tiles of both
    // kinds run side by side and overlap.  (Sorted by cost alone, the large
    // streaming tiles all came first and the Monte-Carlo tiles bunched later;
    // on the 4096-task uneven batch the mix took 651 us against 498 us for
    // its streaming part alone.)
    auto work = [&](uint32_t i) { return (double)tasks[i].n * (double)per_elem(i); };
    uint32_t nm = 0, na = 0;
    double tot_mem = 0, tot_alu = 0;
    for (uint32_t k = 0; k < ntasks; ++k) {
        const uint32_t i = order[k];
        if (tasks[i].kernel_id == SPARKCL_MC_PI) {
            alu[na++] = i;
            tot_alu += work(i);
        } else {
            mem[nm++] = i;
            tot_mem += work(i);
        }
    }
    uint64_t at = 0;
    uint32_t im = 0, ia = 0;
    double done_mem = 0, done_alu = 0;
    while (im < nm || ia < na) {
        const bool take_mem =
            ia == na || (im < nm && done_mem * tot_alu <= done_alu * tot_mem);
        const uint32_t i = take_mem ? mem[im++] : alu[ia++];
        (take_mem ? done_mem : done_alu) += work(i);
        for (uint32_t j = 0; j < dev[i].ntiles; ++j)
            tiles[at++] = TileRef{i, j};
    }
}

int sparkcl::build_plan(sparkcl_ctx *ctx, int kind, int mode, const sparkcl_task *tasks,
                        uint32_t ntasks, sparkcl_result *ures, sparkcl_result *utot,
                        hipStream_t stream, Plan **out, uint32_t per_cu)
{
    std::unique_ptr<Plan> p(new Plan);
    p->kind = kind;
    p->mode = mode;
    p->tasks.assign(tasks, tasks + ntasks);
    p->user_results = ures;
    p->user_total = utot;
    p->ntasks = ntasks;
    p->ntiles.resize(ntasks);
    p->variants.resize(ntasks);

    // Host-input partitions (all or none of the call's tasks) are streamed
    // through staging slots, one per-launch kernel each.
    const bool host_in = kind == 0 && ntasks > 0 && (tasks[0].flags & SPARKCL_TASK_HOST_INPUT);
    for (uint32_t i = 0; i < ntasks; ++i)
        if (((tasks[i].flags & SPARKCL_TASK_HOST_INPUT) != 0) != host_in)
            return fail(SPARKCL_EINVAL, kind == 0 ? "a call's tasks must be all host-input or all device-input"
                                                  : "maps take device arrays");
    p->host = host_in;
    if (host_in && mode == SPARKCL_GRAPH)
        return fail(SPARKCL_EINVAL, "host-input tasks run in PER_LAUNCH or BATCHED mode");
    const Cut cut = plan_cut(ctx, mode, tasks, ntasks, host_in, per_cu);
    p->cut = cut;
    std::vector<uint64_t> first(ntasks);
    std::vector<uint32_t> tile(ntasks);
    uint64_t total_tiles = 0;
    uint32_t kid_mask = 0;
    for (uint32_t i = 0; i < ntasks; ++i) {
        uint32_t v = 0;
        int rc = check_task(tasks[i], &v);
        if (rc != SPARKCL_OK)
            return fail(rc, "task " + std::to_string(i) + ": " + sparkcl_last_error());
        // selective execution: a declined task keeps one empty tile, whose
        // result carries SPARKCL_EDECLINED (maps are never declined)
        const bool skip = kind == 0 && declined(ctx, tasks[i]);
        if (skip)
            v = V_DECLINED;
        p->variants[i] = v;
        const uint32_t T = cut_tile(ctx, cut, tasks[i]);
        tile[i] = T;
        const uint64_t nt = skip ? 1 : std::max<uint64_t>(1, (tasks[i].n + T - 1) / T);
        if (nt > 0xFFFFFFFFull)
            return fail(SPARKCL_ETOOBIG, "too many tiles in task " + std::to_string(i));
        p->ntiles[i] = (uint32_t)nt;
        kid_mask |= 1u << (tasks[i].kernel_id - 1);
        first[i] = total_tiles;
        total_tiles += nt;
    }
    if (total_tiles > 0xFFFFFFF0ull)
        return fail(SPARKCL_ETOOBIG, "too many tiles in one call");
    p->ntiles_total = (uint32_t)total_tiles;

    void *m = nullptr;
    int rc;
#define ALLOC(field, bytes)                                                    \
    do {                                                                       \
        if ((rc = arena_alloc(ctx, p.get(), (bytes), &m)) != SPARKCL_OK) {    \
            for (uint64_t off : p->blocks)                                     \
                ctx->arena.release(off);                                       \
            return rc;                                                         \
        }                                                                      \
        p->field = reinterpret_cast<decltype(p->field)>(m);                    \
    } while (0)
    ALLOC(dtasks, sizeof(TaskDev) * ntasks);
    if (kind == 0) {
        ALLOC(dparts, sizeof(Partial) * total_tiles);
        ALLOC(dsync, sizeof(TaskSync) * ntasks);
        ALLOC(dctl, sizeof(BatchCtl));
        // the RDD total right after the per-task results, so that a blocking
        // call brings both back in one copy
        ALLOC(dresults, sizeof(sparkcl_result) * ((uint64_t)ntasks + 1));
        p->dtotal = p->dresults + ntasks;
        if (mode != SPARKCL_PER_LAUNCH && !host_in)
            ALLOC(dtiles, sizeof(TileRef) * total_tiles);
    }
    if (host_in) {
        // Staging ring: each slot holds one partition's x and y, each placed
        // at the host array's offset modulo 16 bytes so the kernel sees the
        // same quad alignment (and cuts the same tiles) as on the host.
        uint64_t slot = 256;
        for (uint32_t i = 0; i < ntasks; ++i) {
            const uint64_t xb = (tasks[i].n * 4 + 16 + 255) / 256 * 256;
            const uint64_t yb = tasks[i].kernel_id == SPARKCL_FMUL ? xb : 0;
            slot = std::max(slot, xb + yb);
        }
        if (slot > (1ull << 30))
            return fail(SPARKCL_ETOOBIG, "a host-input partition exceeds the 1 GiB staging slot");
        p->nslots = std::min<uint32_t>(ntasks, kStagingSlots);
        p->slot_bytes = slot;
        ALLOC(staging, slot * p->nslots);
    }
#undef ALLOC

    std::vector<TaskDev> host(ntasks);
    for (uint32_t i = 0; i < ntasks; ++i) {
        const sparkcl_task &t = tasks[i];
        TaskDev &d = host[i];
        fill_taskdev(t, p->variants[i], tile[i], p->ntiles[i], i,
                     p->dparts ? p->dparts + first[i] : nullptr,
                     kernel_unroll(ctx->tuning, t.kernel_id), &d);
        if (host_in) {
            char *base = p->staging + (uint64_t)(i % p->nslots) * p->slot_bytes;
            d.in0 = reinterpret_cast<const float *>(base + ((uintptr_t)t.in0 & 15u));
            const uint64_t xb = (t.n * 4 + 16 + 255) / 256 * 256;
            d.in1 = t.kernel_id == SPARKCL_FMUL
                        ? reinterpret_cast<const float *>(base + xb + ((uintptr_t)t.in1 & 15u))
                        : nullptr;
        }
    }
    hipError_t e = hipMemcpyAsync(p->dtasks, host.data(), sizeof(TaskDev) * ntasks,
                                  hipMemcpyHostToDevice, stream);
    std::vector<TileRef> tiles;
    if (e == hipSuccess && p->dtiles) {
        tiles.resize(total_tiles);
        std::vector<uint32_t> order(ntasks), mem(ntasks), alu(ntasks);
        queue_tiles(tasks, ntasks, host.data(), order.data(), mem.data(), alu.data(),
                    tiles.data());
        e = hipMemcpyAsync(p->dtiles, tiles.data(), sizeof(TileRef) * total_tiles,
                           hipMemcpyHostToDevice, stream);
    }
    if (e == hipSuccess && kind == 0) {
        if ((rc = launch_zero(p->dsync, sizeof(TaskSync) * ntasks, stream)) != SPARKCL_OK ||
            (rc = launch_zero(p->dctl, sizeof(BatchCtl), stream)) != SPARKCL_OK)
            e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        for (uint64_t off : p->blocks)
            ctx->arena.release(off);
        return fail_hip(e, "plan upload");
    }

    if (kind == 0) {
        p->out.sync = p->dsync;
        p->out.ctl = p->dctl;
        p->out.results = ures ? ures : p->dresults;
        p->out.total = utot ? utot : p->dtotal;
        // The RDD-level step (one memory-side atomic per finished task, all
        // on one counter) runs only when the total is wanted: an
        // asynchronous call that names per-task results but no total skips
        // it.  Blocking calls (ures == NULL) always return the total.
        p->out.ntasks = (ures && !utot) ? 0 : ntasks;
        p->out.ns_per_tick = ctx->ns_per_tick;
        // map chains run 256-thread blocks; a given per_cu (chains) counts them
        p->block = kind == 4 ? (uint32_t)kBlock : exec_block(ctx, kid_mask);
        p->mc_only = mc_instance(ctx, kid_mask);
        p->grid = std::min(per_cu ? per_cu * (uint32_t)ctx->cus
                                  : exec_grid(ctx, kid_mask, p->ntiles_total, ntasks, p->block),
                           p->ntiles_total);
    }
    if (host_in) {
        p->ev_copied.assign(p->nslots, nullptr);
        p->ev_copied2.assign(p->nslots, nullptr);
        p->ev_done.assign(p->nslots, nullptr);
        hipError_t ee = hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming);
        for (uint32_t k = 0; k < p->nslots && ee == hipSuccess; ++k) {
            ee = hipEventCreateWithFlags(&p->ev_copied[k], hipEventDisableTiming);
            if (ee == hipSuccess)
                ee = hipEventCreateWithFlags(&p->ev_copied2[k], hipEventDisableTiming);
            if (ee == hipSuccess)
                ee = hipEventCreateWithFlags(&p->ev_done[k], hipEventDisableTiming);
        }
        if (ee != hipSuccess) {
            Plan *raw = p.release();
            free_plan(ctx, raw);
            return fail_hip(ee, "staging events");
        }
    }
    p->hash = plan_hash(kind, mode, tasks, ntasks, ures, utot);
    *out = p.release();
    return SPARKCL_OK;
}

int sparkcl::get_plan(sparkcl_ctx *ctx, int kind, int mode, const sparkcl_task *tasks,
                      uint32_t ntasks, sparkcl_result *ures, sparkcl_result *utot,
                      hipStream_t stream, Plan **out)
{
    // fast path: the most recently used plan (a replayed batch) by content
    if (!ctx->plans.empty()) {
        Plan *p = ctx->plans.front();
        if (p->kind == kind && p->mode == mode && p->ntasks == ntasks &&
            p->user_results == ures && p->user_total == utot &&
            std::memcmp(p->tasks.data(), tasks, sizeof(sparkcl_task) * ntasks) == 0) {
            *out = p;
            return SPARKCL_OK;
        }
    }
    const uint64_t h = plan_hash(kind, mode, tasks, ntasks, ures, utot);
    for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it) {
        Plan *p = *it;
        if (p->hash == h && p->kind == kind && p->mode == mode && p->ntasks == ntasks &&
            p->user_results == ures && p->user_total == utot &&
            std::memcmp(p->tasks.data(), tasks, sizeof(sparkcl_task) * ntasks) == 0) {
            ctx->plans.splice(ctx->plans.begin(), ctx->plans, it);
            *out = p;
            return SPARKCL_OK;
        }
    }
    if (capturing(stream))
        return fail(SPARKCL_EINVAL, "no cached plan for this call on a stream under capture: "
                                    "make the same call once before capturing");
    while (ctx->plans.size() >= kMaxPlans)
        evict_one(ctx);
    Plan *p = nullptr;
    int rc = build_plan(ctx, kind, mode, tasks, ntasks, ures, utot, stream, &p);
    if (rc != SPARKCL_OK)
        return rc;
    ctx->plans.push_front(p);
    *out = p;
    return SPARKCL_OK;
}

void sparkcl::drop_plans(sparkcl_ctx *ctx)
{
    (void)hipDeviceSynchronize();
    for (Plan *p : ctx->plans)
        free_plan(ctx, p);
    ctx->plans.clear();
}

int sparkcl::ensure_pinned(sparkcl_ctx *ctx, uint32_t count)
{
    if (count <= ctx->pinned_cap)
        return SPARKCL_OK;
    uint32_t cap = std::max(count, ctx->pinned_cap * 2);
    if (ctx->pinned)
        (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_cap = 0;
    SPARKCL_HIP(hipHostMalloc((void **)&ctx->pinned, sizeof(sparkcl_result) * cap,
                              hipHostMallocDefault));
    ctx->pinned_cap = cap;
    return SPARKCL_OK;
}


bool sparkcl::capturing(hipStream_t stream)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

namespace {

// The kernel launches of a device-input kind-0 plan.
int launch_device(sparkcl_ctx *ctx, Plan *p, hipStream_t stream)
{
    if (p->mode != SPARKCL_PER_LAUNCH) {
        // One dispatch of the persistent executor: the cached plan holds the
        // uploaded task table and tile queue, and the kernel leaves its queue
        // head and tickets at zero, so nothing is cleared between launches.
        int rc = launch_batch(p->dtasks, p->dtiles, p->ntiles_total, p->grid, p->out, stream,
                              p->block, p->mc_only);
        if (rc != SPARKCL_OK)
            return fail(rc, "executor launch failed: " +
                                std::string(hipGetErrorString(hipGetLastError())));
        return SPARKCL_OK;
    }
    for (uint32_t i = 0; i < p->ntasks; ++i) {
        const uint32_t kmask = 1u << (p->tasks[i].kernel_id - 1);
        const uint32_t cap = exec_grid(ctx, kmask);
        int rc = launch_task(p->dtasks + i, p->ntiles[i], std::min(cap, p->ntiles[i]),
                             p->out, stream, exec_block(ctx, kmask));
        if (rc != SPARKCL_OK)
            return fail(rc, "kernel launch failed: " +
                                std::string(hipGetErrorString(hipGetLastError())));
    }
    return SPARKCL_OK;
}

} // namespace

// Enqueue the launches of a reduce-kind plan on `stream`, bracketed by the
// context's timing events.
int sparkcl::enqueue(sparkcl_ctx *ctx, Plan *p, hipStream_t stream, bool timed)
{
    // Timed launches are bracketed by two events (each an extra packet on the
    // queue, a few microseconds apiece), so only blocking calls and the
    // autotuner ask for them; asynchronous calls enqueue the kernels alone.
    if (timed)
        SPARKCL_HIP(hipEventRecord(ctx->ev0, stream));
    if (p->kind == 4) {
        // map chains: the persistent executor over the plan's batched tile
        // queue, with the plan's stage table
        int rc = launch_chain(p->dtasks, p->dtiles, p->ntiles_total, p->dchain, p->grid, p->out,
                              p->chain_unroll,
                              stream);
        if (rc != SPARKCL_OK)
            return fail(rc, "chain launch failed: " +
                                std::string(hipGetErrorString(hipGetLastError())));
    } else if (p->host) {
        if (capturing(stream))
            return fail(SPARKCL_EINVAL, "host-input tasks cannot be captured into a graph");
        // Staged pipeline: partition i is copied into slot i mod S once the
        // kernel that last used the slot is done, and its kernel runs on
        // `stream` once the copies are done.  The x arrays go through one
        // copy stream and the y arrays through another: a stream of copies
        // alternating between the two host arrays moved 2 GiB in 46 ms, two
        // streams each walking one array in 37.7 ms (a single 2 GiB copy:
        // 37.3 ms).  The first copies wait for everything already queued on
        // `stream` (an earlier launch of this plan may still read the slots).
        hipStream_t cs[2] = {ctx->copy_stream, ctx->copy_stream2};
        SPARKCL_HIP(hipEventRecord(p->ev_start, stream));
        for (hipStream_t c : cs)
            SPARKCL_HIP(hipStreamWaitEvent(c, p->ev_start, 0));
        for (uint32_t i = 0; i < p->ntasks; ++i) {
            const sparkcl_task &t = p->tasks[i];
            const uint32_t k = i % p->nslots;
            const bool two = t.kernel_id == SPARKCL_FMUL;
            char *base = p->staging + (uint64_t)k * p->slot_bytes;
            for (int a = 0; a < (two ? 2 : 1); ++a) {
                if (i >= p->nslots)
                    SPARKCL_HIP(hipStreamWaitEvent(cs[a], p->ev_done[k], 0));
                if (t.n) {
                    const void *src = a == 0 ? t.in0 : t.in1;
                    const uint64_t at = a == 0 ? 0 : (t.n * 4 + 16 + 255) / 256 * 256;
                    SPARKCL_HIP(hipMemcpyAsync(base + at + ((uintptr_t)src & 15u), src,
                                               t.n * 4, hipMemcpyHostToDevice, cs[a]));
                }
                hipEvent_t ev = a == 0 ? p->ev_copied[k] : p->ev_copied2[k];
                SPARKCL_HIP(hipEventRecord(ev, cs[a]));
                SPARKCL_HIP(hipStreamWaitEvent(stream, ev, 0));
            }
            const uint32_t kmask = 1u << (t.kernel_id - 1);
            const uint32_t cap = exec_grid(ctx, kmask);
            int rc = launch_task(p->dtasks + i, p->ntiles[i], std::min(cap, p->ntiles[i]),
                                 p->out, stream, exec_block(ctx, kmask));
            if (rc != SPARKCL_OK)
                return fail(rc, "kernel launch failed: " +
                                    std::string(hipGetErrorString(hipGetLastError())));
            SPARKCL_HIP(hipEventRecord(p->ev_done[k], stream));
        }
    } else if (p->mode == SPARKCL_GRAPH && !capturing(stream)) {
        // The launches below, captured once on the library's own stream into
        // a graph kept with the plan, then replayed: one graph launch per
        // call.  Under the caller's capture they are recorded directly.
        if (!p->gexec[0]) {
            hipStream_t cs = ctx->capture_stream;
            SPARKCL_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            const int rc = launch_device(ctx, p, cs);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(cs, &g);
            if (rc != SPARKCL_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess)
                return fail_hip(e, "graph capture");
            hipGraphExec_t x[2] = {nullptr, nullptr};
            for (hipGraphExec_t &e : x) {
                const hipError_t ei = hipGraphInstantiateWithFlags(&e, g, 0);
                if (ei != hipSuccess) {
                    if (x[0])
                        (void)hipGraphExecDestroy(x[0]);
                    (void)hipGraphDestroy(g);
                    return fail_hip(ei, "graph instantiate");
                }
            }
            p->graph = g;
            p->gexec[0] = x[0];
            p->gexec[1] = x[1];
        }
        // the two instances take turns (a launch waits for its instance's
        // previous launch; the other instance's is then one call back)
        SPARKCL_HIP(hipGraphLaunch(p->gexec[p->glaunches++ & 1u], stream));
    } else {
        const int rc = launch_device(ctx, p, stream);
        if (rc != SPARKCL_OK)
            return rc;
    }
    if (timed) {
        SPARKCL_HIP(hipEventRecord(ctx->ev1, stream));
        ctx->have_ms = true;
    }
    if (p->kind == 0) {
        sparkcl_launch_shape &s = ctx->shape;
        s = sparkcl_launch_shape{};
        const bool per_task = p->mode == SPARKCL_PER_LAUNCH || p->host;
        uint32_t kmask = 0;
        for (const sparkcl_task &t : p->tasks)
            kmask |= 1u << (t.kernel_id - 1);
        s.grid = per_task ? 0 : p->grid;
        // per-task launches take each kernel's own block size
        s.block = per_task && (kmask & (kmask - 1)) ? 0 : p->block;
        s.ntiles = p->ntiles_total;
        s.ntasks = p->ntasks;
        s.tile_table = p->cut.tm == TM_BATCHED ? 1 : 0;
        s.mixed = p->cut.mixed ? 1 : 0;
        s.mode = (uint32_t)p->mode;
        for (uint32_t k = 0; k < 3 && p->cut.mixed; ++k)
            s.mixed_tile[k] = ctx->tuning.tile_many[k]
                                  ? ctx->tuning.tile_many[k]
                                  : p->cut.share_tile[k];
        ctx->have_shape = true;
    }
    return SPARKCL_OK;
}

int sparkcl::launch_and_collect(sparkcl_ctx *ctx, Plan *p, const sparkcl_task *tasks,
                                uint32_t ntasks, sparkcl_result *per_task,
                                sparkcl_result *total, hipStream_t stream)
{
    int rc;
    if ((rc = ensure_pinned(ctx, ntasks + 1)) != SPARKCL_OK)
        return rc;
    if ((rc = enqueue(ctx, p, stream, true)) != SPARKCL_OK)
        return rc;
    // the per-task results and the RDD total behind them, in one copy
    SPARKCL_HIP(hipMemcpyAsync(ctx->pinned, p->dresults,
                               sizeof(sparkcl_result) * ((uint64_t)ntasks + 1),
                               hipMemcpyDeviceToHost, stream));
    SPARKCL_HIP(hipStreamSynchronize(stream));
    if (per_task)
        std::memcpy(per_task, ctx->pinned, sizeof(sparkcl_result) * ntasks);
    if (total) {
        *total = ctx->pinned[ntasks];
        uint32_t ops = 0;
        for (uint32_t i = 0; i < ntasks; ++i)
            ops |= tasks[i].reduce_ops;
        if (!(ops & SPARKCL_SUM))
            total->sum = 0.0;
        if (!(ops & SPARKCL_MAX))
            total->max = -__builtin_huge_valf();
        if (!(ops & SPARKCL_COUNT))
            total->count = 0;
    }
    return SPARKCL_OK;
}

int sparkcl::check_ctx(sparkcl_ctx *ctx)
{
    if (!ctx)
        return fail(SPARKCL_EINVAL, "null context");
    SPARKCL_HIP(hipSetDevice(ctx->device));
    return SPARKCL_OK;
}

namespace {

// The caller holds ctx->mu.
int run_blocking_locked(sparkcl_ctx *ctx, int mode, const sparkcl_task *tasks,
                        uint32_t ntasks, sparkcl_result *per_task, sparkcl_result *total,
                        hipStream_t stream)
{
    Plan *p = nullptr;
    int rc = get_plan(ctx, 0, mode, tasks, ntasks, nullptr, nullptr, stream, &p);
    if (rc != SPARKCL_OK)
        return rc;
    return launch_and_collect(ctx, p, tasks, ntasks, per_task, total, stream);
}

int run_blocking(sparkcl_ctx *ctx, int mode, const sparkcl_task *tasks,
                 uint32_t ntasks, sparkcl_result *per_task, sparkcl_result *total,
                 hipStream_t stream)
{
    if (capturing(stream))
        return fail(SPARKCL_EINVAL, "a blocking call cannot run on a stream under capture");
    std::lock_guard<std::mutex> g(ctx->mu);
    return run_blocking_locked(ctx, mode, tasks, ntasks, per_task, total, stream);
}

} // namespace

extern "C" {

const char *sparkcl_version(void) { return "sparkcl-mi355x 0.1"; }

const char *sparkcl_strerror(int code)
{
    switch (code) {
    case SPARKCL_OK: return "ok";
    case SPARKCL_EINVAL: return "invalid argument";
    case SPARKCL_ENOKERNEL: return "kernel id not in the registry";
    case SPARKCL_ETOOBIG: return "task too big";
    case SPARKCL_EAGAIN: return "not ready";
    case SPARKCL_EHIP: return "HIP runtime error";
    case SPARKCL_ETIMEDOUT: return "timed out";
    case SPARKCL_ESTOPPED: return "stopped";
    case SPARKCL_ENOMEM: return "arena exhausted";
    case SPARKCL_ENOTFOUND: return "unknown ticket";
    case SPARKCL_EDECLINED: return "declined by selective execution";
    default: return "unknown status";
    }
}

const char *sparkcl_last_error(void) { return t_last_error.c_str(); }

int sparkcl_init(const sparkcl_config *config, sparkcl_ctx **out)
{
    if (!out)
        return fail(SPARKCL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!config)
        return fail(SPARKCL_EINVAL, "config is NULL");
    int ndev = 0;
    SPARKCL_HIP(hipGetDeviceCount(&ndev));
    if (config->device < 0 || config->device >= ndev)
        return fail(SPARKCL_EINVAL, "device " + std::to_string(config->device) +
                                        " out of range (" + std::to_string(ndev) + ")");
    uint32_t cap = config->ring_capacity ? config->ring_capacity : 4096;
    if (cap & (cap - 1) || cap > (1u << 20))
        return fail(SPARKCL_EINVAL, "ring_capacity must be a power of two <= 2^20");
    uint64_t arena_bytes = config->arena_bytes ? config->arena_bytes : (256ull << 20);
    if (arena_bytes < (16ull << 20))
        return fail(SPARKCL_EINVAL, "arena_bytes below 16 MiB");
    if (config->arena && ((uintptr_t)config->arena & 255u))
        return fail(SPARKCL_EINVAL, "arena must be 256-byte aligned");

    std::unique_ptr<sparkcl_ctx> ctx(new sparkcl_ctx);
    ctx->config = *config;
    ctx->config.ring_capacity = cap;
    ctx->config.arena_bytes = arena_bytes;
    if (!ctx->config.budget_bytes)
        ctx->config.budget_bytes = arena_bytes;
    if (!ctx->config.idle_exit_ms)
        ctx->config.idle_exit_ms = 1000;
    if (!ctx->config.watchdog_ms)
        ctx->config.watchdog_ms = 10000;
    ctx->device = config->device;
    SPARKCL_HIP(hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    SPARKCL_HIP(hipGetDeviceProperties(&prop, ctx->device));
    ctx->arch = prop.gcnArchName;
    ctx->cus = prop.multiProcessorCount;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device) ==
            hipSuccess &&
        rate_khz > 0)
        ctx->ns_per_tick = std::max(1, 1000000 / rate_khz);
    int occ = 0;
    int rc = batch_blocks_per_cu(&occ);
    if (rc != SPARKCL_OK)
        return fail(rc, "occupancy query failed");
    ctx->occ_batch = std::max(1, occ);
    occ = 0;
    if ((rc = batch_mc_blocks_per_cu(&occ)) != SPARKCL_OK)
        return fail(rc, "occupancy query failed");
    ctx->occ_mc = std::max(1, occ);
    occ = 0;
    if ((rc = chain_blocks_per_cu(&occ)) != SPARKCL_OK)
        return fail(rc, "occupancy query failed");
    ctx->occ_chain = std::max(1, occ);

    tuning_defaults(&ctx->tuning);
    if (config->tune_cache) {
        std::string err;
        sparkcl_tuning t;
        if (tuning_load_file(config->tune_cache, ctx->arch, &t, &err))
            ctx->tuning = t;
        // a missing or foreign cache keeps the defaults
    }

    if (config->arena) {
        ctx->arena_base = static_cast<char *>(config->arena);
    } else {
        SPARKCL_HIP(hipMalloc((void **)&ctx->arena_base, arena_bytes));
        ctx->own_arena = true;
    }
    ctx->arena.reset(arena_bytes);
    SPARKCL_HIP(hipEventCreate(&ctx->ev0));
    SPARKCL_HIP(hipEventCreate(&ctx->ev1));
    SPARKCL_HIP(hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
    SPARKCL_HIP(hipStreamCreateWithFlags(&ctx->copy_stream2, hipStreamNonBlocking));
    SPARKCL_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    if ((rc = ensure_pinned(ctx.get(), 1024)) != SPARKCL_OK)
        return rc;
    if ((rc = noalloc_setup(ctx->device)) != SPARKCL_OK)
        return rc;
    rc = Server::create(ctx.get(), &ctx->server);
    if (rc != SPARKCL_OK)
        return rc;
    *out = ctx.release();
    return SPARKCL_OK;
}

int sparkcl_destroy(sparkcl_ctx *ctx)
{
    if (!ctx)
        return fail(SPARKCL_EINVAL, "null context");
    (void)hipSetDevice(ctx->device);
    int rc = SPARKCL_OK;
    if (ctx->server)
        rc = ctx->server->shutdown();
    ctx->server.reset();
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        drop_plans(ctx);
    }
    if (ctx->pinned)
        (void)hipHostFree(ctx->pinned);
    if (ctx->ev0)
        (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1)
        (void)hipEventDestroy(ctx->ev1);
    if (ctx->copy_stream)
        (void)hipStreamDestroy(ctx->copy_stream);
    if (ctx->copy_stream2)
        (void)hipStreamDestroy(ctx->copy_stream2);
    if (ctx->capture_stream)
        (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->own_arena)
        (void)hipFree(ctx->arena_base);
    delete ctx;
    return rc;
}

int sparkcl_map(sparkcl_ctx *ctx, const sparkcl_task *tasks, uint32_t ntasks, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (ntasks && !tasks)
        return fail(SPARKCL_EINVAL, "tasks is NULL");
    for (uint32_t i = 0; i < ntasks; ++i) {
        if (tasks[i].kernel_id == SPARKCL_MC_PI)
            return fail(SPARKCL_EINVAL, "MC_PI is a partition kernel, not a map");
        if (tasks[i].n && !tasks[i].out)
            return fail(SPARKCL_EINVAL, "map needs an output array");
    }
    if (ntasks == 0)
        return SPARKCL_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Plan *p = nullptr;
    if ((rc = get_plan(ctx, 1, 0, tasks, ntasks, nullptr, nullptr, s, &p)) != SPARKCL_OK)
        return rc;
    const uint32_t cap = (uint32_t)ctx->occ_batch * (uint32_t)ctx->cus;
    for (uint32_t i = 0; i < ntasks; ++i) {
        const uint64_t n = tasks[i].n;
        if (n == 0)
            continue;
        const uint64_t want = (n / 4 + kBlock - 1) / kBlock;
        const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, cap));
        if ((rc = launch_map(p->dtasks + i, n, p->variants[i], grid, s)) != SPARKCL_OK)
            return fail(rc, "map launch failed");
    }
    return SPARKCL_OK;
}

int sparkcl_map_partition(sparkcl_ctx *ctx, const sparkcl_task *tasks, uint32_t ntasks,
                          int mode, sparkcl_result *results, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (ntasks && (!tasks || !results))
        return fail(SPARKCL_EINVAL, "tasks/results is NULL");
    if (mode != SPARKCL_PER_LAUNCH && mode != SPARKCL_BATCHED && mode != SPARKCL_GRAPH)
        return fail(SPARKCL_EINVAL, "unknown mode");
    for (uint32_t i = 0; i < ntasks; ++i)
        if (tasks[i].kernel_id != SPARKCL_MC_PI)
            return fail(tasks[i].kernel_id >= 1 && tasks[i].kernel_id <= 3 ? SPARKCL_EINVAL
                                                                            : SPARKCL_ENOKERNEL,
                        "map_partition runs partition kernels (MC_PI)");
    if (ntasks == 0)
        return SPARKCL_OK;
    return run_blocking(ctx, mode, tasks, ntasks, results, nullptr,
                        static_cast<hipStream_t>(stream));
}

int sparkcl_reduce(sparkcl_ctx *ctx, const sparkcl_task *tasks, uint32_t ntasks, int mode,
                   sparkcl_result *per_task, sparkcl_result *total, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (ntasks && !tasks)
        return fail(SPARKCL_EINVAL, "tasks is NULL");
    if (mode != SPARKCL_PER_LAUNCH && mode != SPARKCL_BATCHED && mode != SPARKCL_GRAPH)
        return fail(SPARKCL_EINVAL, "unknown mode");
    if (ntasks == 0) {
        if (total) {
            std::memset(total, 0, sizeof(*total));
            total->max = -__builtin_huge_valf();
        }
        return SPARKCL_OK;
    }
    return run_blocking(ctx, mode, tasks, ntasks, per_task, total,
                        static_cast<hipStream_t>(stream));
}

int sparkcl_reduce_async(sparkcl_ctx *ctx, const sparkcl_task *tasks, uint32_t ntasks,
                         int mode, sparkcl_result *dev_per_task, sparkcl_result *dev_total,
                         void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (ntasks == 0)
        return SPARKCL_OK;
    if (!tasks)
        return fail(SPARKCL_EINVAL, "tasks is NULL");
    if (mode != SPARKCL_PER_LAUNCH && mode != SPARKCL_BATCHED && mode != SPARKCL_GRAPH)
        return fail(SPARKCL_EINVAL, "unknown mode");
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Plan *p = nullptr;
    if ((rc = get_plan(ctx, 0, mode, tasks, ntasks, dev_per_task, dev_total, s, &p)) !=
        SPARKCL_OK)
        return rc;
    return enqueue(ctx, p, s, false);
}

int sparkcl_offload_breakeven(sparkcl_ctx *ctx, double host_bytes_per_s, uint64_t *bytes)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (!bytes || !(host_bytes_per_s > 0.0))
        return fail(SPARKCL_EINVAL, "bytes is NULL or the host rate is not positive");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!(ctx->offload_gpu_bps > 0.0)) {
        // Measured with the threshold off: the fixed cost is the median host
        // time of a blocking reduce of one element; the streaming rate comes
        // from a blocking reduce of 2^26 floats (256 MiB) less that cost.
        constexpr uint64_t kElems = 1ull << 26;
        const uint64_t off = ctx->arena.alloc(kElems * 4);
        if (off == Arena::kFail)
            return fail(SPARKCL_ENOMEM, "offload measurement needs 256 MiB of free arena");
        float *buf = static_cast<float *>(ctx->dev(off));
        const uint64_t saved = ctx->config.offload_min_bytes;
        ctx->config.offload_min_bytes = 0;
        auto once = [&](uint64_t n, double *sec) -> int {
            sparkcl_task t;
            std::memset(&t, 0, sizeof(t));
            t.kernel_id = SPARKCL_POLY;
            t.reduce_ops = SPARKCL_SUM;
            t.n = n;
            t.in0 = buf;
            sparkcl_result r;
            const uint64_t t0 = host_ns();
            int e = run_blocking_locked(ctx, SPARKCL_BATCHED, &t, 1, &r, nullptr, nullptr);
            *sec = (double)(host_ns() - t0) * 1e-9;
            return e;
        };
        auto median = [&](uint64_t n, int reps, double *sec) -> int {
            std::vector<double> v(reps);
            for (int i = 0; i < reps; ++i) {
                int e = once(n, &v[i]);
                if (e != SPARKCL_OK)
                    return e;
            }
            std::sort(v.begin(), v.end());
            *sec = v[reps / 2];
            return SPARKCL_OK;
        };
        double fixed = 0, big = 0;
        rc = launch_zero(buf, kElems * 4, nullptr);
        if (rc == SPARKCL_OK && hipDeviceSynchronize() != hipSuccess)
            rc = SPARKCL_EHIP;
        if (rc == SPARKCL_OK)
            rc = median(1, 15, &fixed);
        if (rc == SPARKCL_OK)
            rc = median(kElems, 7, &big);
        drop_plans(ctx); // the measured plans point into the scratch block
        ctx->arena.release(off);
        ctx->config.offload_min_bytes = saved;
        if (rc != SPARKCL_OK)
            return fail(rc, std::string("offload measurement failed: ") + sparkcl_last_error());
        ctx->offload_fixed_s = fixed;
        ctx->offload_gpu_bps = (double)(kElems * 4) / std::max(big - fixed, 1e-9);
    }
    const double inv = 1.0 / host_bytes_per_s - 1.0 / ctx->offload_gpu_bps;
    if (!(inv > 0.0)) {
        *bytes = UINT64_MAX;
        return SPARKCL_OK;
    }
    const double b = ctx->offload_fixed_s / inv;
    *bytes = b >= 1.8e19 ? UINT64_MAX : (uint64_t)std::ceil(b);
    return SPARKCL_OK;
}

int sparkcl_submit(sparkcl_ctx *ctx, const sparkcl_task *task, uint64_t *ticket)
{
    if (!ctx || !ctx->server)
        return fail(SPARKCL_EINVAL, "null context");
    if (!task || !ticket)
        return fail(SPARKCL_EINVAL, "task/ticket is NULL");
    return ctx->server->submit(*task, ticket);
}

int sparkcl_poll(sparkcl_ctx *ctx, uint64_t ticket, sparkcl_result *result)
{
    if (!ctx || !ctx->server)
        return fail(SPARKCL_EINVAL, "null context");
    if (!result)
        return fail(SPARKCL_EINVAL, "result is NULL");
    return ctx->server->poll(ticket, result);
}

int sparkcl_serve_stats_get(sparkcl_ctx *ctx, sparkcl_serve_stats *stats)
{
    if (!ctx || !ctx->server || !stats)
        return fail(SPARKCL_EINVAL, "null argument");
    ctx->server->stats(stats);
    return SPARKCL_OK;
}

int sparkcl_serve_drain(sparkcl_ctx *ctx, uint32_t timeout_ms)
{
    if (!ctx || !ctx->server)
        return fail(SPARKCL_EINVAL, "null context");
    return ctx->server->drain(timeout_ms);
}

int sparkcl_get_tuning(sparkcl_ctx *ctx, sparkcl_tuning *out)
{
    if (!ctx || !out)
        return fail(SPARKCL_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    *out = ctx->tuning;
    return SPARKCL_OK;
}

int sparkcl_set_tuning(sparkcl_ctx *ctx, const sparkcl_tuning *in)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    std::string why;
    if (tuning_validate(in, &why) != SPARKCL_OK)
        return fail(SPARKCL_EINVAL, why);
    std::lock_guard<std::mutex> g(ctx->mu);
    drop_plans(ctx);
    ctx->tuning = *in;
    if (ctx->server)
        ctx->server->set_tuning(*in);
    return SPARKCL_OK;
}

int sparkcl_last_launch_shape(sparkcl_ctx *ctx, sparkcl_launch_shape *out)
{
    if (!ctx || !out)
        return fail(SPARKCL_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!ctx->have_shape)
        return fail(SPARKCL_EAGAIN, "no reduce-kind call yet");
    *out = ctx->shape;
    return SPARKCL_OK;
}

int sparkcl_last_kernel_ms(sparkcl_ctx *ctx, float *ms)
{
    if (!ctx || !ms)
        return fail(SPARKCL_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!ctx->have_ms)
        return fail(SPARKCL_EAGAIN, "no launch timed yet");
    SPARKCL_HIP(hipEventSynchronize(ctx->ev1));
    SPARKCL_HIP(hipEventElapsedTime(ms, ctx->ev0, ctx->ev1));
    return SPARKCL_OK;
}

} // extern "C"
