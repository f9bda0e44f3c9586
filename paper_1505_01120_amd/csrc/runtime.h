// Internal runtime types shared by the C ABI (api.cpp, arrays.cpp, chain.cpp,
// wordcount.cpp) and the serving loop (serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "arena.h"
#include "sparkcl.h"
#include "sparkcl_dev.h"
#include "tuning.h"

namespace sparkcl {

// Sets this thread's sparkcl_last_error() text and returns `code`.
int fail(int code, const std::string &msg);
int fail_hip(hipError_t e, const char *what);

#define SPARKCL_HIP(expr)                                                      \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::sparkcl::fail_hip(e_, #expr);                             \
    } while (0)

// Validates one task and derives its kernel body selector.
int check_task(const sparkcl_task &t, uint32_t *variant);
// Selective execution: a task's offload cost in bytes, and whether the
// context's threshold declines it.
uint64_t offload_cost(const sparkcl_task &t);
// Input bytes a streaming kernel reads per element (x, and y for FMUL).
uint64_t input_bytes(uint32_t kernel_id);
bool declined(const sparkcl_ctx *ctx, const sparkcl_task &t);

// Host steady-clock time in ns.
uint64_t host_ns();

class Server;

// How a reduce-kind call is cut into tiles: the tuning table's row (batched
// or per-launch) and whether the mixed-batch tile sizes apply.
struct Cut {
    int tm = TM_PER_LAUNCH;
    bool mixed = false;
    // mixed batches: each kernel's tile derived from the batch's totals and
    // the tuned tiles per CU (index kernel id - 1; 0: none derived)
    uint32_t share_tile[3] = {0, 0, 0};
};

// A cached, uploaded launch: device task table, tile queue, partials, sync
// words and results.
struct Plan {
    uint64_t hash = 0;
    int kind = 0; // 0 reduce/map_partition, 1 map, 2/3 array reduce (table/rows), 4 chain
    int mode = 0;
    std::vector<sparkcl_task> tasks;
    sparkcl_result *user_results = nullptr;
    sparkcl_result *user_total = nullptr;

    std::vector<uint64_t> blocks; // arena offsets owned
    TaskDev *dtasks = nullptr;
    TileRef *dtiles = nullptr;
    Partial *dparts = nullptr;
    TaskSync *dsync = nullptr;
    BatchCtl *dctl = nullptr;
    sparkcl_result *dresults = nullptr;
    sparkcl_result *dtotal = nullptr;
    uint32_t ntasks = 0;
    uint32_t ntiles_total = 0;
    std::vector<uint32_t> ntiles;
    std::vector<uint32_t> variants;
    uint32_t grid = 0;
    uint32_t block = 256; // executor threads per block
    bool mc_only = false; // every task Monte-Carlo: the executor's MC instance
    Cut cut{};            // kind 0: the tile table the call was cut with
    LaunchOut out{};

    // kinds 2 and 3, array-valued ReduceCL: the leaves (a pointer table, or
    // rows of one buffer) and the passes
    uint32_t combiner = 0;
    uint64_t len = 0;
    float *user_out = nullptr;
    bool vec4 = false;
    uint32_t nleaves = 0;
    const float *leaf_base = nullptr;
    uint64_t leaf_stride = 0;
    std::vector<const float *> leaves;
    std::vector<TreeArgs> passes;

    // kind 4, map chains: the stage table and the loads in flight
    ChainDev chain{};
    ChainDev *dchain = nullptr;
    uint32_t chain_unroll = 4;

    // host-input partitions: the staging ring and its events
    bool host = false;
    uint32_t nslots = 0;
    uint64_t slot_bytes = 0;
    char *staging = nullptr;
    hipEvent_t ev_start = nullptr;
    std::vector<hipEvent_t> ev_copied, ev_copied2, ev_done; // x copied, y copied, slot free

    // SPARKCL_GRAPH: the plan's launches captured once, replayed per call.
    // Two executable instances of the graph take turns: the runtime makes a
    // launch of an instance wait until that instance's previous launch has
    // finished, so with one instance a replayed call could not be queued
    // behind the one still running, and the GPU idled between them.
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    uint32_t glaunches = 0;
};

// Plan cache and launch helpers (api.cpp); the caller holds ctx->mu.
constexpr uint32_t kMaxPlans = 32;     // cached plans per context
// A batched call is "mixed" (takes sparkcl_tuning.tile_many) with at least
// this many tasks whose sizes span at least this many log2 buckets.
constexpr uint32_t kMixedMinTasks = 512;
constexpr uint32_t kMixedMinSpan = 4;
constexpr uint64_t kMaxN = 1ull << 40; // elements (or samples, bytes) per task

// Plan cache helpers (api.cpp); the caller holds ctx->mu.
uint64_t fnv1a(uint64_t h, const void *p, size_t n);
uint64_t plan_hash(int kind, int mode, const sparkcl_task *tasks, uint32_t ntasks,
                   const void *ures, const void *utot);
void free_plan(sparkcl_ctx *ctx, Plan *p);
// Evicts the least recently used plan (after a device-wide wait); false if
// no plan is left.
bool evict_one(sparkcl_ctx *ctx);
// Arena block for plan p, evicting older plans while the arena is full.
int arena_alloc(sparkcl_ctx *ctx, Plan *p, uint64_t bytes, void **out);
// The cut of a call: a function of the call, the tuning table and the
// executor occupancy; allocates nothing.
Cut plan_cut(const sparkcl_ctx *ctx, int mode, const sparkcl_task *tasks, uint32_t ntasks,
             bool host_in, uint32_t per_cu = 0);
// The tile size of one task under a cut.
uint32_t cut_tile(const sparkcl_ctx *ctx, const Cut &c, const sparkcl_task &t);
// The device descriptor of one task.
void fill_taskdev(const sparkcl_task &t, uint32_t variant, uint32_t tile, uint32_t ntiles,
                  uint32_t index, Partial *partials, uint32_t unroll, TaskDev *d);
// The batched tile queue (longest first, streaming and Monte-Carlo tiles
// interleaved) into tiles[sum of dev[i].ntiles]; order, mem and alu are
// caller-provided arrays of ntasks entries.  Allocates nothing.
void queue_tiles(const sparkcl_task *tasks, uint32_t ntasks, const TaskDev *dev,
                 uint32_t *order, uint32_t *mem, uint32_t *alu, TileRef *tiles);
// A reduce-kind plan (kind 0) for the call; per_cu: executor blocks per CU
// (0: the tuned choice).
int build_plan(sparkcl_ctx *ctx, int kind, int mode, const sparkcl_task *tasks,
               uint32_t ntasks, sparkcl_result *ures, sparkcl_result *utot,
               hipStream_t stream, Plan **out, uint32_t per_cu = 0);
// Launches plan p (timed) and copies its results to host memory.
int launch_and_collect(sparkcl_ctx *ctx, Plan *p, const sparkcl_task *tasks,
                       uint32_t ntasks, sparkcl_result *per_task, sparkcl_result *total,
                       hipStream_t stream);
// A non-null context, made current on this thread.
int check_ctx(sparkcl_ctx *ctx);
// Pinned host staging for at least `count` results.
int ensure_pinned(sparkcl_ctx *ctx, uint32_t count);

// A call on a stream under capture may only reuse a cached plan: building
// one uploads and synchronises, which a capture cannot hold.
int get_plan(sparkcl_ctx *ctx, int kind, int mode, const sparkcl_task *tasks,
             uint32_t ntasks, sparkcl_result *ures, sparkcl_result *utot,
             hipStream_t stream, Plan **out);
bool capturing(hipStream_t stream);
int enqueue(sparkcl_ctx *ctx, Plan *p, hipStream_t stream, bool timed);
void drop_plans(sparkcl_ctx *ctx);
// Allocation-free workspace (noalloc.hip): looks up this device's address of
// the fixed device array once per device; `device` must be current.
int noalloc_setup(int device);
// Persistent-executor grid for a batch holding the kernels in kid_mask
// (bit k-1 for kernel id k) and `ntiles` tiles over `ntasks` tasks.
uint32_t exec_grid(const sparkcl_ctx *ctx, uint32_t kid_mask, uint64_t ntiles = 0,
                   uint64_t ntasks = 0, uint32_t block = 0);
// The executor's threads per block for a batch holding the kernels in
// kid_mask (one kernel: its tuned size; several: the mixed-batch size), and
// the float4 loads in flight per thread for a kernel's streaming loop.
uint32_t exec_block(const sparkcl_ctx *ctx, uint32_t kid_mask);
// Executor blocks per CU that fit for a batch holding the kernels in
// kid_mask (the Monte-Carlo-only instance fits more).
uint32_t exec_occupancy(const sparkcl_ctx *ctx, uint32_t kid_mask);
// Whether a batch holding the kernels in kid_mask runs the Monte-Carlo-only
// executor instance (Monte-Carlo tasks alone).
bool mc_instance(const sparkcl_ctx *ctx, uint32_t kid_mask);
uint32_t kernel_unroll(const sparkcl_tuning &t, uint32_t kid);

} // namespace sparkcl

struct sparkcl_ctx {
    int device = 0;
    std::string arch;
    int cus = 0;
    uint32_t ns_per_tick = 10;
    int occ_batch = 1; // batch-executor blocks per CU that fit
    int occ_mc = 1;    // blocks per CU of the Monte-Carlo-only executor
    // autotuner only: Monte-Carlo batches run the shared executor, so that
    // blocks_per_cu[MC_PI] is measured where mixed batches use it
    bool tune_shared_mc = false;
    int occ_chain = 1; // chain-executor blocks per CU that fit
    int occ_wordcount = 0; // word-count blocks per CU that fit (0: not yet asked)

    char *arena_base = nullptr;
    bool own_arena = false;
    sparkcl::Arena arena;

    sparkcl_tuning tuning{};
    sparkcl_config config{};

    std::mutex mu; // plans, events, pinned buffers
    std::list<sparkcl::Plan *> plans; // most recently used first
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t copy_stream = nullptr;  // host-input staging copies of x
    hipStream_t copy_stream2 = nullptr; // and of y
    hipStream_t capture_stream = nullptr; // builds SPARKCL_GRAPH plans' graphs
    bool have_ms = false;
    bool have_shape = false;
    sparkcl_launch_shape shape{}; // of the last reduce-kind call
    double offload_fixed_s = 0.0;   // selective execution: measured fixed
    double offload_gpu_bps = 0.0;   // cost and streaming rate (0: not yet)
    sparkcl_result *pinned = nullptr;
    uint32_t pinned_cap = 0;

    std::unique_ptr<sparkcl::Server> server;

    void *dev(uint64_t off) const { return arena_base + off; }
};
