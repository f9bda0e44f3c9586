// Allocation-free ReduceCL: the batched launch of sparkcl_reduce_async (one
// persistent-executor dispatch over a device tile queue; ReduceCL, sec.
// 3.1.3) with every workspace it needs -- task table, tile queue, partials,
// arrival tickets, queue counters and internal results -- in one fixed array
// of device memory instead of blocks of the context's arena, for callers that
// cannot allocate.  The decomposition is the same function of the call, the
// tuning table and the occupancy as in sparkcl_reduce_async, so the results
// are bit-identical to it.
//
// The array is a file-scope __device__ object: each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never names it directly (in host code its name is a host-side stand-in, not
// a device address): at context set-up the device address is looked up once
// per device with hipGetSymbolAddress and kept, and kernels and copies get
// that address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "runtime.h"

namespace sparkcl {

namespace {

constexpr uint32_t kMaxTasks = SPARKCL_NOALLOC_MAX_TASKS;
constexpr uint32_t kMaxTiles = SPARKCL_NOALLOC_MAX_TILES;
constexpr int kMaxDevices = 64;

// Regions of the array (byte offsets, each 256-byte aligned).
constexpr uint64_t kOffCtl = 0;       // BatchCtl: queue head, exit count, RDD ticket
constexpr uint64_t kOffTotal = 256;   // RDD total when the caller passes none
constexpr uint64_t kOffTasks = 512;   // TaskDev[kMaxTasks]
constexpr uint64_t kOffSync = kOffTasks + sizeof(TaskDev) * (uint64_t)kMaxTasks;
constexpr uint64_t kOffResults = kOffSync + sizeof(TaskSync) * (uint64_t)kMaxTasks;
constexpr uint64_t kOffTiles = kOffResults + sizeof(sparkcl_result) * (uint64_t)kMaxTasks;
constexpr uint64_t kOffParts = kOffTiles + sizeof(TileRef) * (uint64_t)kMaxTiles;
constexpr uint64_t kScratchBytes = kOffParts + sizeof(Partial) * (uint64_t)kMaxTiles;
static_assert(kScratchBytes == SPARKCL_NOALLOC_SCRATCH_BYTES, "header states the size");
static_assert(kOffSync % 256 == 0 && kOffResults % 256 == 0 && kOffTiles % 256 == 0 &&
                  kOffParts % 256 == 0,
              "regions stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    char *ptr = nullptr;       // this device's address of `scratch`
    hipEvent_t done = nullptr; // recorded after each call's launches on this device
};
DeviceScratch g_dev[kMaxDevices];

// One call at a time in the process: the host staging below is shared, and
// a call waits for the previous call's work (g_last) before it rewrites the
// staging or a device's array.
std::mutex g_mu;
hipEvent_t g_last = nullptr;

// Host staging of the uploaded tables (static storage, not allocated per call).
TaskDev h_tasks[kMaxTasks];
TileRef h_tiles[kMaxTiles];
uint32_t h_order[kMaxTasks], h_mem[kMaxTasks], h_alu[kMaxTasks];

} // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return SPARKCL_OK; // allocation-free calls refuse this device (EINVAL)
    std::lock_guard<std::mutex> g(g_mu);
    DeviceScratch &d = g_dev[device];
    if (d.ptr)
        return SPARKCL_OK;
    // the caller (sparkcl_init) has made `device` current
    void *ptr = nullptr;
    SPARKCL_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
    if (!ptr)
        return fail(SPARKCL_EHIP, "allocation-free workspace: no device address");
    hipEvent_t e = nullptr;
    SPARKCL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    d.ptr = static_cast<char *>(ptr);
    d.done = e;
    return SPARKCL_OK;
}

} // namespace sparkcl

using namespace sparkcl;

extern "C" int sparkcl_reduce_noalloc(sparkcl_ctx *ctx, const sparkcl_task *tasks,
                                      uint32_t ntasks, sparkcl_result *dev_per_task,
                                      sparkcl_result *dev_total, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (ntasks == 0)
        return SPARKCL_OK;
    if (!tasks)
        return fail(SPARKCL_EINVAL, "tasks is NULL");
    if (ntasks > kMaxTasks)
        return fail(SPARKCL_ETOOBIG, "allocation-free reduce takes at most " +
                                         std::to_string(kMaxTasks) + " tasks");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (capturing(s))
        return fail(SPARKCL_EINVAL, "allocation-free reduce cannot run under stream capture");
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_dev[ctx->device].ptr)
        return fail(SPARKCL_EINVAL, "no allocation-free workspace on device " +
                                        std::to_string(ctx->device));
    std::lock_guard<std::mutex> g(g_mu);
    DeviceScratch &dv = g_dev[ctx->device];
    char *base = dv.ptr;
    // The previous call's kernels (any stream, any device) may still read the
    // staging's upload or their device's array: wait for them before either
    // is rewritten.
    if (g_last)
        SPARKCL_HIP(hipEventSynchronize(g_last));

    // Decompose exactly as the batched sparkcl_reduce_async does.
    Cut cut;
    uint64_t total_tiles = 0;
    uint32_t kid_mask = 0, grid = 0, block = 256;
    {
        std::lock_guard<std::mutex> gc(ctx->mu); // tuning table, threshold
        for (uint32_t i = 0; i < ntasks; ++i) {
            if (tasks[i].flags & SPARKCL_TASK_HOST_INPUT)
                return fail(SPARKCL_EINVAL, "allocation-free reduce takes device inputs");
            uint32_t v = 0;
            if ((rc = check_task(tasks[i], &v)) != SPARKCL_OK)
                return fail(rc, "task " + std::to_string(i) + ": " + sparkcl_last_error());
        }
        cut = plan_cut(ctx, SPARKCL_BATCHED, tasks, ntasks, false);
        for (uint32_t i = 0; i < ntasks; ++i) {
            const uint32_t T = cut_tile(ctx, cut, tasks[i]);
            const bool skip = declined(ctx, tasks[i]);
            total_tiles += skip ? 1 : std::max<uint64_t>(1, (tasks[i].n + T - 1) / T);
            kid_mask |= 1u << (tasks[i].kernel_id - 1);
        }
        if (total_tiles > kMaxTiles)
            return fail(SPARKCL_ETOOBIG, "allocation-free reduce takes at most " +
                                             std::to_string(kMaxTiles) + " tiles, the call needs " +
                                             std::to_string(total_tiles));
        grid = std::min<uint64_t>(exec_grid(ctx, kid_mask, total_tiles, ntasks), total_tiles);
        block = exec_block(ctx, kid_mask);

        Partial *parts = reinterpret_cast<Partial *>(base + kOffParts);
        uint64_t first = 0;
        for (uint32_t i = 0; i < ntasks; ++i) {
            uint32_t v = 0;
            (void)check_task(tasks[i], &v);
            const bool skip = declined(ctx, tasks[i]);
            if (skip)
                v = V_DECLINED;
            const uint32_t T = cut_tile(ctx, cut, tasks[i]);
            const uint32_t nt =
                skip ? 1u : (uint32_t)std::max<uint64_t>(1, (tasks[i].n + T - 1) / T);
            fill_taskdev(tasks[i], v, T, nt, i, parts + first,
                         kernel_unroll(ctx->tuning, tasks[i].kernel_id), &h_tasks[i]);
            first += nt;
        }
    }
    queue_tiles(tasks, ntasks, h_tasks, h_order, h_mem, h_alu, h_tiles);

    BatchCtl *ctl = reinterpret_cast<BatchCtl *>(base + kOffCtl);
    TaskSync *sync = reinterpret_cast<TaskSync *>(base + kOffSync);
    TaskDev *dtasks = reinterpret_cast<TaskDev *>(base + kOffTasks);
    TileRef *dtiles = reinterpret_cast<TileRef *>(base + kOffTiles);
    SPARKCL_HIP(hipMemcpyAsync(dtasks, h_tasks, sizeof(TaskDev) * ntasks,
                               hipMemcpyHostToDevice, s));
    SPARKCL_HIP(hipMemcpyAsync(dtiles, h_tiles, sizeof(TileRef) * total_tiles,
                               hipMemcpyHostToDevice, s));
    // The array keeps the last call's contents: the arrival tickets, start
    // times and queue counters must start at zero (a fill kernel, no memset).
    if ((rc = launch_zero(sync, sizeof(TaskSync) * ntasks, s)) != SPARKCL_OK ||
        (rc = launch_zero(ctl, sizeof(BatchCtl), s)) != SPARKCL_OK)
        return fail(rc, "clearing the allocation-free workspace failed");
    LaunchOut L{};
    L.sync = sync;
    L.ctl = ctl;
    L.results = dev_per_task ? dev_per_task
                             : reinterpret_cast<sparkcl_result *>(base + kOffResults);
    L.total = dev_total ? dev_total : reinterpret_cast<sparkcl_result *>(base + kOffTotal);
    // as sparkcl_reduce_async: per-task results and no total skip the fold
    L.ntasks = (dev_per_task && !dev_total) ? 0 : ntasks;
    L.ns_per_tick = ctx->ns_per_tick;
    if ((rc = launch_batch(dtasks, dtiles, (uint32_t)total_tiles, grid, L, s, block,
                           mc_instance(ctx, kid_mask))) != SPARKCL_OK)
        return fail(rc, "executor launch failed: " +
                            std::string(hipGetErrorString(hipGetLastError())));
    SPARKCL_HIP(hipEventRecord(dv.done, s));
    g_last = dv.done;
    return SPARKCL_OK;
}
