// ReduceCL over fused map chains (sec. 3.1.3: a map is pipelined into the
// action that consumes it): each task's registry map followed by up to
// kMaxPost POLY stages, reduced in one pass of the persistent executor.
#include <algorithm>
#include <cstring>
#include <string>

#include "runtime.h"

using namespace sparkcl;

extern "C" {

int sparkcl_reduce_chain(sparkcl_ctx *ctx, const sparkcl_task *tasks, uint32_t ntasks,
                         const sparkcl_stage *stages, uint32_t nstages,
                         sparkcl_result *per_task, sparkcl_result *total, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if ((ntasks && !tasks) || (nstages && !stages))
        return fail(SPARKCL_EINVAL, "tasks/stages is NULL");
    if (nstages > (uint32_t)kMaxPost)
        return fail(SPARKCL_EINVAL, "more than " + std::to_string(kMaxPost) + " chain stages");
    ChainDev chain;
    std::memset(&chain, 0, sizeof(chain));
    chain.npost = nstages;
    for (uint32_t s = 0; s < nstages; ++s) {
        if (stages[s].kernel_id != SPARKCL_POLY || stages[s].degree > 7)
            return fail(SPARKCL_EINVAL, "chain stage " + std::to_string(s) +
                                            " must be POLY of degree <= 7");
        chain.deg[s] = stages[s].degree;
        std::memcpy(chain.coef[s], stages[s].coef, sizeof(chain.coef[s]));
    }
    for (uint32_t i = 0; i < ntasks; ++i)
        if (tasks[i].kernel_id == SPARKCL_MC_PI || (tasks[i].flags & SPARKCL_TASK_HOST_INPUT))
            return fail(SPARKCL_EINVAL, "map chains take POLY/FMUL tasks with device inputs");
    if (ntasks == 0)
        return SPARKCL_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (capturing(st))
        return fail(SPARKCL_EINVAL, "a blocking call cannot run on a stream under capture");
    const uint64_t h = fnv1a(plan_hash(4, SPARKCL_BATCHED, tasks, ntasks, nullptr, nullptr),
                             &chain, sizeof(chain));
    Plan *p = nullptr;
    for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it) {
        Plan *q = *it;
        if (q->kind == 4 && q->hash == h && q->ntasks == ntasks &&
            std::memcmp(q->tasks.data(), tasks, sizeof(sparkcl_task) * ntasks) == 0 &&
            std::memcmp(&q->chain, &chain, sizeof(chain)) == 0) {
            ctx->plans.splice(ctx->plans.begin(), ctx->plans, it);
            p = q;
            break;
        }
    }
    if (!p) {
        while (ctx->plans.size() >= kMaxPlans)
            evict_one(ctx);
        // The chain's Horner steps add dependent VALU work per element, whose
        // latency either more waves per CU or more loads in flight per wave
        // hide.  Measured on MI355X (64 x 2^22 FMUL partitions): no steps
        // streams best at the map's tuned occupancy (1 block per CU, 316 us);
        // 3 steps with 8 float4 loads in flight per thread and input at 1
        // block per CU (324 us; with 4 loads: 346-351 at 2 blocks per CU,
        // 354-359 at 3, 397-408 at 1); 28 steps (four degree-7 stages) with
        // 4 loads at 4 blocks per CU (407-411 us; with 8 loads 526-558 at 3,
        // where the deeper stream's registers cap the waves).  A grid that
        // would get fewer than two of the batched table's tiles per block
        // takes the per-launch table's smaller tiles, so blocks keep pulling
        // tiles from the queue (with one large tile per block, blocks placed
        // unevenly on the CUs decide the time: 440-490 us at 2 per CU).
        uint32_t steps = 0;
        for (uint32_t s = 0; s < nstages; ++s)
            steps += chain.deg[s];
        uint32_t base = 0;
        for (uint32_t i = 0; i < ntasks; ++i)
            if (tasks[i].kernel_id == SPARKCL_POLY)
                base = std::max(base, tasks[i].degree);
        steps += base;
        const bool deep = steps >= 1 && steps <= 4;
        uint32_t per_cu = 0;
        if (!ctx->config.exec_blocks_per_cu) {
            const uint32_t want = steps == 0 ? 0 : deep ? 1 : steps <= 12 ? 3 : 4;
            per_cu = std::min(want, (uint32_t)ctx->occ_chain);
        }
        if ((rc = build_plan(ctx, 0, SPARKCL_BATCHED, tasks, ntasks, nullptr, nullptr, st,
                             &p, per_cu)) != SPARKCL_OK)
            return rc;
        p->kind = 4;
        p->chain = chain;
        p->chain_unroll = deep ? 8 : 4;
        p->hash = h;
        void *d = nullptr;
        if ((rc = arena_alloc(ctx, p, sizeof(ChainDev), &d)) != SPARKCL_OK) {
            free_plan(ctx, p);
            return rc;
        }
        p->dchain = static_cast<ChainDev *>(d);
        hipError_t e = hipMemcpyAsync(d, &p->chain, sizeof(ChainDev), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_plan(ctx, p);
            return fail_hip(e, "chain upload");
        }
        ctx->plans.push_front(p);
    }
    return launch_and_collect(ctx, p, tasks, ntasks, per_task, total, st);
}

} // extern "C"
