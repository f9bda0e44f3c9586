/*
 * sparkcl.h -- C ABI of the SparkCL map -> reduce offload hot path on MI355X.
 *
 * The paper's model (SparkCL, sec. 3.1): a user kernel is applied to the data of
 * RDD partitions through three constructs (sec. 3.1.3):
 *   MapCL          -- elementwise kernel over a partition        -> sparkcl_map
 *   MapCLPartition -- kernel over a whole partition              -> sparkcl_map_partition
 *   ReduceCL       -- kernel-driven reduction, tree-combined      -> sparkcl_reduce
 * The paper's SparkKernel (Fig 2) bundles a data-preparation hook, the kernel
 * body and a result hook; here a task descriptor (sparkcl_task) carries what
 * mapParameters prepares (data, range, parameters), a registry kernel id names
 * the body, and sparkcl_result is what mapReturnValue hands back.  Java kernels
 * cannot be compiled here, so a registry of three built-in kernels stands in
 * for user kernels:
 *   SPARKCL_POLY  -- y = sum_k coef[k] x^k (Horner, degree <= 7), one input
 *   SPARKCL_FMUL  -- z = x*y + c*x, two inputs (the SparkKernel2 arity of Fig 3)
 *   SPARKCL_MC_PI -- Philox4x32-10 Monte-Carlo quarter-disc hit count
 *                    (the SparkCLPi demo, sec. 3.2.1)
 *
 * Conventions for every entry point:
 *   - Returns SPARKCL_OK (0) or a negative SPARKCL_E* code; nothing throws
 *     across the ABI.  sparkcl_last_error() gives this thread's detail text.
 *   - Input/output arrays named "device" are device pointers owned by the
 *     caller; they must stay valid until the call returns (blocking calls),
 *     until the stream reaches the work (async calls), or until sparkcl_poll
 *     reports the task done (serving).
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *   - Floating point: maps evaluate each multiply and add as one binary32
 *     operation in the order written (no contraction), so materialised map
 *     outputs are bit-exact.  Sums are accumulated per thread in FP64 and
 *     combined in FP64 across the wave, the block and the partition's tiles,
 *     and returned as double.  For a
 *     given context and inputs every result is run-to-run identical.
 *   - An empty partition (n == 0) gives sum +0.0, max -inf, count 0.
 */
#ifndef SPARKCL_H
#define SPARKCL_H

#include <stdint.h>

#if defined(__GNUC__)
#define SPARKCL_API __attribute__((visibility("default")))
#else
#define SPARKCL_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SPARKCL_OK 0
#define SPARKCL_EINVAL (-1)    /* bad argument: NULL with n > 0, bad op mask,
                                  degree > 7, wrong kernel for the call ...  */
#define SPARKCL_ENOKERNEL (-2) /* kernel id not in the registry               */
#define SPARKCL_ETOOBIG (-3)   /* task bytes exceed the serving budget, or a
                                  size beyond the library's limits            */
#define SPARKCL_EAGAIN (-4)    /* serving: not done yet / queue full          */
#define SPARKCL_EHIP (-5)      /* a HIP runtime call failed (see last_error)  */
#define SPARKCL_ETIMEDOUT (-6) /* a bounded wait expired                      */
#define SPARKCL_ESTOPPED (-7)  /* serving stopped / context being destroyed   */
#define SPARKCL_ENOMEM (-8)    /* arena exhausted for library workspaces      */
#define SPARKCL_ENOTFOUND (-9) /* unknown serving ticket                      */
#define SPARKCL_EDECLINED (-10) /* selective execution: the task is below the
                                   context's offload threshold and was not
                                   run; run the host function for it         */

/* ---- registry ---------------------------------------------------------- */
#define SPARKCL_POLY 1
#define SPARKCL_FMUL 2
#define SPARKCL_MC_PI 3

/* reduce-op bits: POLY/FMUL accept a non-empty subset of SUM|MAX; MC_PI
   accepts COUNT only. */
#define SPARKCL_SUM 1u
#define SPARKCL_MAX 2u
#define SPARKCL_COUNT 4u

/* combiners of the array-valued ReduceCL (sparkcl_reduce_arrays) */
#define SPARKCL_VADD 1u /* c[i] = a[i] + b[i], one binary32 add (Fig 3)     */
#define SPARKCL_VMAX 2u /* c[i] = (b[i] > a[i]) ? b[i] : a[i]                 */

/* execution modes of sparkcl_reduce / sparkcl_map_partition */
#define SPARKCL_PER_LAUNCH 0 /* one kernel launch per partition              */
#define SPARKCL_BATCHED 1    /* all partitions in one persistent launch over
                                a device tile queue (cached per call content) */
#define SPARKCL_GRAPH 2      /* the BATCHED launch captured once into a
                                hipGraph kept with the cached plan, and
                                replayed on every later call with the same
                                content (device-resident inputs only) */

typedef struct sparkcl_ctx sparkcl_ctx; /* opaque, library-owned */

/* sparkcl_config.flags bits */
#define SPARKCL_FLAG_SERVE_PER_TASK 1u /* serving runs one kernel launch per
                                         task over a pool of 4 streams (the
                                         one-task-at-a-time baseline) instead
                                         of the resident executor            */

/* Context configuration.  Zero fields take the defaults shown. */
typedef struct sparkcl_config {
    int32_t device;             /* HIP device ordinal                        */
    uint32_t ring_capacity;     /* serving slots (tasks on the device at
                                   once), power of two; 0 -> 4096            */
    void *arena;                /* device memory the library sub-allocates
                                   for every workspace it needs (tile
                                   queues, partials, tickets, results);
                                   caller-owned, valid until destroy.  The
                                   library calls no hipMalloc after init.    */
    uint64_t arena_bytes;       /* size of `arena`; at least 16 MiB          */
    uint64_t budget_bytes;      /* serving admission budget (input + output
                                   + partial bytes of tasks on the device);
                                   0 -> arena_bytes                          */
    uint32_t exec_blocks_per_cu;/* persistent executor blocks per CU; 0 ->
                                   tuned value                               */
    uint32_t idle_exit_ms;      /* resident serving executor exits after this
                                   long with no work (relaunched on demand);
                                   0 -> 1000                                 */
    uint32_t watchdog_ms;       /* serving: a task not done this long after
                                   admission is failed with ETIMEDOUT; 0 ->
                                   10000                                     */
    uint32_t flags;             /* SPARKCL_FLAG_* bits                       */
    const char *tune_cache;     /* JSON tuning cache (tile sizes per kernel
                                   and size bucket, keyed by gfx arch); NULL
                                   -> built-in defaults                      */
    uint64_t offload_min_bytes; /* selective execution (sec. 3.1.1: the
                                   kernel may decline accelerated execution
                                   and mapReturnValue then calls an
                                   alternative function): a task whose
                                   offload cost -- bytes read, 4n for POLY,
                                   8n for FMUL; 4n for MC_PI, whose sample
                                   costs about as much GPU time as 4 bytes of
                                   streaming -- is below this is declined:
                                   not run, result status SPARKCL_EDECLINED
                                   with sum +0, max -inf, count 0, n 0 (so it
                                   adds nothing to the RDD total); submit
                                   returns SPARKCL_EDECLINED.  0 -> never.
                                   sparkcl_offload_breakeven suggests one.   */
} sparkcl_config;

/* One partition task: what mapParameters prepares in the paper (Fig 2, Fig 3):
   the data arrays, the range (n) and the kernel's parameters. */
typedef struct sparkcl_task {
    uint32_t kernel_id;    /* SPARKCL_POLY / SPARKCL_FMUL / SPARKCL_MC_PI   */
    uint32_t reduce_ops;   /* SPARKCL_SUM | SPARKCL_MAX | SPARKCL_COUNT      */
    uint64_t n;            /* elements (POLY, FMUL) or samples (MC_PI)       */
    const float *in0;      /* device x[n] (POLY, FMUL); any 4-byte alignment */
    const float *in1;      /* device y[n] (FMUL)                             */
    float *out;            /* device map output [n] or NULL (POLY, FMUL)     */
    uint64_t seed;         /* MC_PI: Philox key = (seed lo, seed hi)         */
    uint32_t partition_id; /* MC_PI: Philox counter word 2                   */
    uint32_t degree;       /* POLY: 0..7                                     */
    float coef[8];         /* POLY: coef[k] multiplies x^k                   */
    float c;               /* FMUL constant                                  */
    uint32_t flags;        /* SPARKCL_TASK_* bits; 0 for device inputs       */
} sparkcl_task;

/* sparkcl_task.flags: in0 / in1 are HOST arrays (POLY, FMUL; out must be
   NULL).  sparkcl_reduce / sparkcl_reduce_async then stream the partitions
   through a ring of device staging slots in the arena: the host-to-device
   copy of partition i+1 (on the library's copy stream) overlaps the kernel of
   partition i, each partition one kernel launch cut by the per-launch tile
   table, whatever `mode` says.  A call's tasks are all host or all device.
   Host arrays must stay valid until the call's results are ready; pinned
   memory (hipHostMalloc) overlaps, pageable memory works but copies
   synchronously.  Each partition's input bytes must fit one staging slot
   (ETOOBIG beyond 1 GiB).  Results are bit-identical to the same data
   reduced from device memory in SPARKCL_PER_LAUNCH mode.
   Served (sparkcl_submit) host-input tasks must use pinned host memory
   (EINVAL otherwise): the server charges the task's staging block (its
   inputs, each at its host address modulo 16, in 256-byte units) and
   partials against the budget, copies the inputs into the arena on its own
   copy streams while other tasks run, and hands the task to the executor
   once the copy is done; its latency includes the transfer.  Its result is
   bit-identical to the same data served from device memory at the same
   16-byte alignment.  ETOOBIG if the staging block exceeds the arena. */
#define SPARKCL_TASK_HOST_INPUT 1u

/* What mapReturnValue hands back for one partition (or the RDD total). */
typedef struct sparkcl_result {
    double sum;            /* SUM requested: FP64 sum, else +0.0              */
    float max;             /* MAX requested: max, else -inf                   */
    int32_t status;        /* SPARKCL_OK or the task's error                  */
    uint64_t count;        /* COUNT: hits (MC_PI), else 0                     */
    uint64_t n;            /* elements/samples covered by the tiles           */
    uint64_t t_arrive_ns;  /* serving: submit time (host steady clock)        */
    uint64_t t_admit_ns;   /* serving: admission time (host steady clock)     */
    uint64_t t_start_ns;   /* first tile started (device clock, 10 ns steps)  */
    uint64_t t_done_ns;    /* serving: completion seen (host steady clock);
                              batch: last tile done (device clock)            */
} sparkcl_result;

/* Create a context on config->device.  Validates the config, loads tuning,
   allocates the host-coherent serving ring (pinned host memory) and carves
   its workspaces out of config->arena.  *out is NULL on error.  The paper
   leaves memory allocation to the framework rather than to the user's
   algorithm (sec. 3, design issue 3): every workspace of every later call is
   sub-allocated from the arena handed over here, so no call allocates device
   memory.  The kernels themselves are compiled into the library and loaded
   once per context, the paper's kernel caching per worker (sec. 3.1.1.2). */
SPARKCL_API int sparkcl_init(const sparkcl_config *config, sparkcl_ctx **out);

/* Stop serving (waits up to 10 s for the resident executor to drain), release
   pinned memory and cached plans.  The arena itself stays the caller's. */
SPARKCL_API int sparkcl_destroy(sparkcl_ctx *ctx);

/* MapCL (sec. 3.1.3): out[i] = kernel(in0[i] [, in1[i]]) for each task
   (POLY or FMUL, out != NULL).  Asynchronous on `stream`; bit-exact against
   the binary32 definition.  reduce_ops is ignored. */
SPARKCL_API int sparkcl_map(sparkcl_ctx *ctx, const sparkcl_task *tasks, uint32_t ntasks,
                void *stream);

/* MapCLPartition (sec. 3.1.3): run a partition kernel (MC_PI, ops COUNT) on
   each task and write one partition-level result per task into results[]
   (host memory, ntasks entries).  mode: SPARKCL_PER_LAUNCH,
   SPARKCL_BATCHED or SPARKCL_GRAPH.  Blocking. */
SPARKCL_API int sparkcl_map_partition(sparkcl_ctx *ctx, const sparkcl_task *tasks,
                          uint32_t ntasks, int mode, sparkcl_result *results,
                          void *stream);

/* ReduceCL (sec. 3.1.3, tree-reduce; sec. 3.2.2): for each task, the map fused
   with the requested reductions (no intermediate array unless task.out is
   set, in which case the map output is also written), then the RDD-level
   combine of all partition results in task order.  per_task (ntasks entries)
   and total are host memory; either may be NULL.  Blocking. */
SPARKCL_API int sparkcl_reduce(sparkcl_ctx *ctx, const sparkcl_task *tasks,
                   uint32_t ntasks, int mode, sparkcl_result *per_task,
                   sparkcl_result *total, void *stream);

/* The same as sparkcl_reduce without the host synchronisation: results are
   written by the GPU to dev_per_task[ntasks] and *dev_total (device memory,
   caller-owned; either may be NULL; with dev_per_task set and dev_total NULL
   the RDD-level total is not computed) in stream order.  Calls that share a
   context must not overlap in time on different streams.
   Stream capture: a call on a stream that is being captured into the
   caller's own graph records the plan's launches into that graph, with no
   memset nodes (the executor leaves its queue head and tickets at zero for
   the next replay).  The plan must already be cached, so make the same call
   once outside the capture first; otherwise, and for host-input tasks, the
   call returns SPARKCL_EINVAL.  With SPARKCL_GRAPH under capture the plan's
   launches are recorded directly instead of nesting its graph. */
SPARKCL_API int sparkcl_reduce_async(sparkcl_ctx *ctx, const sparkcl_task *tasks,
                         uint32_t ntasks, int mode,
                         sparkcl_result *dev_per_task,
                         sparkcl_result *dev_total, void *stream);

/* One stage of a fused map chain: a registry map applied to the running
   value of the chain.  Stages are POLY (kernel_id SPARKCL_POLY, degree 0..7,
   coef[k] multiplies v^k). */
typedef struct sparkcl_stage {
    uint32_t kernel_id;
    uint32_t degree;
    float coef[8];
} sparkcl_stage;

/* ReduceCL over fused map chains (a Spark stage: map -> map -> ... ->
   reduce, pipelined in one pass; sec. 3.1.3): each task's own map (POLY or
   FMUL, with its parameters) is followed by the `nstages` stages in order,
   each evaluated one binary32 multiply and add per Horner step with no
   contraction, then the task's reductions; task.out, if set, receives the
   chain's final values (bit-exact).  At most 4 stages; MC_PI and host-input
   tasks are rejected (EINVAL).  All partitions run in one persistent launch
   over the batched tile queue, as SPARKCL_BATCHED; per_task / total as in
   sparkcl_reduce.  Blocking. */
SPARKCL_API int sparkcl_reduce_chain(sparkcl_ctx *ctx, const sparkcl_task *tasks,
                                     uint32_t ntasks, const sparkcl_stage *stages,
                                     uint32_t nstages, sparkcl_result *per_task,
                                     sparkcl_result *total, void *stream);

/* Array-valued ReduceCL (sec. 3.1.3 item 3; the Fig 3 vector add; sec.
   3.2.2): the RDD's elements are `k` float arrays of `len` elements each, in
   RDD order; arrays[] is a HOST array of k DEVICE pointers (caller-owned, any
   4-byte alignment; with len % 4 == 0 the columns are read as float4).  The combiner (SPARKCL_VADD or SPARKCL_VMAX) folds them pairwise
   along a fixed tree -- over elements [k0, k1) the split is at k0 plus the
   largest power of two below the count, left part the left operand -- and
   the result goes to out[0..len) (device memory; it may be one of the
   inputs).  Bit-exact against that definition.  Asynchronous on `stream`;
   k may not exceed 2^24; intermediate rows (when the reduction runs in
   several passes) come from the arena: ENOMEM if it is too small.  EINVAL
   for k == 0, a NULL pointer, an unknown combiner or a misaligned array. */
SPARKCL_API int sparkcl_reduce_arrays(sparkcl_ctx *ctx, uint32_t combiner,
                                      const float *const *arrays, uint32_t k,
                                      uint64_t len, float *out, void *stream);

/* The same array-valued ReduceCL over RDD elements stored as the rows of one
   device buffer: element e is base[e * row_stride .. e * row_stride + len)
   (row_stride in elements, >= len when k > 1).  No pointer table is built or
   hashed, so very many short elements cost nothing on the host.  Bit-exact
   against the same tree; same errors and stream semantics. */
SPARKCL_API int sparkcl_reduce_rows(sparkcl_ctx *ctx, uint32_t combiner,
                                    const float *base, uint64_t row_stride,
                                    uint32_t k, uint64_t len, float *out,
                                    void *stream);

/* Serving (continuous batching): enqueue one task, stamping its arrival.
   Non-blocking.  The task is admitted to the resident executor once a slot is
   free and its bytes fit the budget; tasks admitted while others run share
   the GPU with them.  *ticket identifies it for sparkcl_poll.  ETOOBIG if the
   task alone exceeds the budget; EAGAIN if the pending queue is full.
   The paper's workers take one accelerated task at a time so that tasks do
   not contend for the device (sec. 3.1.5, Fig 4, `--cores 1`), and note that
   the framework has its own provisions against contention; here that
   provision is admission control: a task is admitted only against a free
   slot and the memory budget (sec. 3, design issue 3), and admitted tasks
   share the GPU's compute units through one resident executor. */
SPARKCL_API int sparkcl_submit(sparkcl_ctx *ctx, const sparkcl_task *task,
                   uint64_t *ticket);

/* Serving: SPARKCL_OK and *result when the task is done (the ticket is then
   retired), SPARKCL_EAGAIN while pending, ENOTFOUND for an unknown ticket.
   A failed task returns OK with result->status holding its error.  This is
   the serving form of mapReturnValue (Fig 2, sec. 3.1.1.3): the partition's
   value, or EDECLINED when the task was not offloaded and the caller's
   alternative must compute it. */
SPARKCL_API int sparkcl_poll(sparkcl_ctx *ctx, uint64_t ticket, sparkcl_result *result);

typedef struct sparkcl_serve_stats {
    uint64_t submitted, admitted, completed, failed;
    uint64_t pending;          /* submitted, not yet admitted               */
    uint64_t in_flight;        /* admitted, not yet complete                */
    uint64_t budget_in_use;    /* bytes charged against the budget          */
    uint64_t budget_peak;
    uint64_t admission_waits;  /* times the queue head waited for budget or
                                  a slot                                    */
    uint64_t executor_launches;/* resident executor (re)launches            */
} sparkcl_serve_stats;

SPARKCL_API int sparkcl_serve_stats_get(sparkcl_ctx *ctx, sparkcl_serve_stats *stats);

/* Wait until every submitted task is complete, up to timeout_ms. */
SPARKCL_API int sparkcl_serve_drain(sparkcl_ctx *ctx, uint32_t timeout_ms);

/* ---- tuning ------------------------------------------------------------ */
#define SPARKCL_TUNE_BUCKETS 32  /* log2(n) buckets 0..31 */
#define SPARKCL_TUNE_MODES 3     /* PER_LAUNCH, BATCHED, serving */

typedef struct sparkcl_tuning {
    uint32_t blocks_per_cu[3];   /* persistent-executor blocks per CU for each
                                    registry kernel (index kernel id - 1); a
                                    batch uses the largest among the kernels
                                    it holds (a batch of Monte-Carlo tasks
                                    alone: blocks_per_cu_mc_only); 0 = as
                                    many as fit                               */
    uint32_t blocks_per_cu_many; /* the executor's blocks per CU for a batch of
                                    many small tasks (under 4 tiles per task
                                    on average), where per-tile latency
                                    rather than streaming depth dominates;
                                    0 = as many as fit                        */
    uint32_t tile_many[3];       /* batched tile size per kernel for a batch of
                                    many tasks of widely spread sizes (at
                                    least 512 tasks whose sizes span 4 or
                                    more log2 buckets), in place of the
                                    per-bucket table: there, small tasks run
                                    best whole and large ones in mid-sized
                                    tiles; 0 = use the table, else a power of
                                    two from 2^10 to 2^22                     */
    uint32_t block[3];           /* threads per block of the batch executor and
                                    the per-partition kernel for each registry
                                    kernel (a batch of one kernel takes its
                                    kernel's; serving, map chains and maps use
                                    256): 256, 512 or 1024; 0 = 256          */
    uint32_t block_many;         /* the executor's block size for a batch that
                                    mixes kernels; 0 = 256                    */
    uint32_t unroll[3];          /* float4 loads in flight per thread and
                                    input in the POLY / FMUL streaming loops
                                    (index kernel id - 1; MC_PI has none):
                                    2, 4 or 8; 0 = 4.  Block size and unroll
                                    fix which thread sums which elements, so
                                    sums are identical across calls that
                                    share them and the tile size.             */
    uint32_t many_tiles_per_cu[2]; /* for such a batch of many spread tasks,
                                    when tile_many leaves a kernel at 0: the
                                    number of tiles per CU to cut the batch's
                                    streaming input bytes [0] (4 per POLY
                                    element, 8 per FMUL element) or its
                                    Monte-Carlo samples [1] into; a kernel's
                                    tile is the batch's total over (CUs x
                                    this value), in its own elements, rounded
                                    to the nearest power of two in
                                    [2^10, 2^22].  A work share, unlike a tile
                                    size, carries over between batches of
                                    different totals.  0 = use the per-bucket
                                    table; else 1 to 4096                     */
    uint32_t blocks_per_cu_mc_only; /* blocks per CU for a batch of Monte-Carlo
                                    tasks alone, which runs an executor
                                    instance holding only the Philox body
                                    (fewer registers, so more blocks fit);
                                    0 = as many as fit, else 1 to 32          */
    /* tile size in elements (samples for MC_PI) for [mode][kernel-1][log2 n];
       powers of two from 2^10 to 2^22.  A batched call whose executor blocks
       would get fewer than two of the batched row's tiles each is cut with
       the per-launch row instead. */
    uint32_t tile[SPARKCL_TUNE_MODES][3][SPARKCL_TUNE_BUCKETS];
} sparkcl_tuning;

SPARKCL_API int sparkcl_get_tuning(sparkcl_ctx *ctx, sparkcl_tuning *out);
/* Replace the tuning table (validated: tiles must be powers of two in range).
   Cached plans are dropped. */
SPARKCL_API int sparkcl_set_tuning(sparkcl_ctx *ctx, const sparkcl_tuning *in);

/* Autotuner (the paper leaves such optimisation open, sec. 6): on synthetic
   device data, by median HIP-event time, with a 2% margin a candidate must
   beat: per kernel, the executor blocks per CU jointly with the tile for
   2^22-element partitions, then blocks per CU, block size and loads in
   flight jointly (and, for Monte-Carlo, the occupancy of the instance that
   runs Monte-Carlo tasks alone); then the tile size per execution mode,
   kernel and size bucket in [lo_log2, hi_log2]; then, on a mixed batch of
   its own distribution, the many-task occupancy, the work shares and the
   mixed-batch block size.  Writes the table into the context and, if
   `path` is non-NULL, into that JSON file under the device's gfx arch name.
   Needs 2 GiB of free arena. */
SPARKCL_API int sparkcl_autotune(sparkcl_ctx *ctx, uint32_t lo_log2, uint32_t hi_log2,
                     const char *path);

/* ---- diagnostics ------------------------------------------------------- */
SPARKCL_API const char *sparkcl_strerror(int code);
SPARKCL_API const char *sparkcl_last_error(void);

/* Device kernel time (ms) of the last blocking reduce/map_partition launch
   sequence on this context, measured with HIP events on the launch stream
   (asynchronous calls are not timed, so they add no event packets). */
SPARKCL_API int sparkcl_last_kernel_ms(sparkcl_ctx *ctx, float *ms);

/* How the last reduce/map_partition call on this context (blocking or
   asynchronous) was cut and launched: the scheduling decisions of sec. 3.1.5
   (how an RDD's partitions are spread over the device) as this library takes
   them from the tuning table.  Written into *out; SPARKCL_EAGAIN before the
   first such call. */
typedef struct sparkcl_launch_shape {
    uint32_t grid;        /* persistent-executor blocks; 0 for PER_LAUNCH
                             (one launch per task) and host-input calls     */
    uint32_t block;       /* threads per executor block; 0 for per-task
                             launches of several kernels (each takes its
                             own tuned size)                                */
    uint32_t ntiles;      /* tiles the call was cut into                    */
    uint32_t ntasks;
    uint32_t tile_table;  /* 0: the per-launch tile table, 1: the batched one */
    uint32_t mixed;       /* 1: cut with the mixed-batch tiles (tile_many or
                             many_tiles_per_cu)                            */
    uint32_t mode;        /* SPARKCL_PER_LAUNCH, _BATCHED or _GRAPH         */
    uint32_t mixed_tile[3]; /* when mixed: each kernel's tile size (index
                             kernel id - 1), 0 where it took the per-bucket
                             table                                          */
} sparkcl_launch_shape;

SPARKCL_API int sparkcl_last_launch_shape(sparkcl_ctx *ctx, sparkcl_launch_shape *out);

/* WordCount (sec. 3.2.3, the Spark word-count demo as a SparkCL kernel) over
   `nbytes` bytes of device text: a word is a maximal run of bytes that are
   not ASCII whitespace (space, tab, LF, VT, FF, CR), counted under the 64-bit
   FNV-1a hash of its bytes.  The distinct keys and their counts go to
   keys[] / counts[] (device arrays of `capacity` entries, caller-owned), in no
   particular order; *ndistinct and *nwords (host) receive the number of
   distinct keys and of words.  Blocking.  The counting table comes from the
   arena (16 B per slot, two slots per key of capacity, at least 1024):
   ENOMEM if it does not fit; ETOOBIG if there are more distinct keys than
   `capacity` (*ndistinct is then at least capacity + 1), or if nbytes
   exceeds 2^40. */
SPARKCL_API int sparkcl_wordcount(sparkcl_ctx *ctx, const uint8_t *text, uint64_t nbytes,
                                  uint64_t *keys, uint64_t *counts, uint64_t capacity,
                                  uint64_t *ndistinct, uint64_t *nwords, void *stream);

/* WordCount's words (sec. 3.2.3 counts words, which sparkcl_wordcount names
   by their keys): for each of the `nkeys` distinct keys in keys[] (device
   memory, e.g. the first *ndistinct entries sparkcl_wordcount wrote), the
   byte offset in the same `nbytes` of device text of the first word whose
   key it is, written to offsets[] (device, nkeys entries, caller-owned);
   UINT64_MAX for a key that no word of the text has.  The word is the run
   of non-whitespace bytes starting there.  One pass over the text plus a
   lookup table from the arena (12 B per slot, two slots per key, at least
   1024): ENOMEM if it does not fit; EINVAL if a key appears twice (offsets
   are then unspecified); ETOOBIG if nkeys exceeds 2^32 - 1 or nbytes
   exceeds 2^40.  Blocking. */
SPARKCL_API int sparkcl_wordcount_locate(sparkcl_ctx *ctx, const uint8_t *text,
                                         uint64_t nbytes, const uint64_t *keys,
                                         uint64_t nkeys, uint64_t *offsets, void *stream);

/* Selective execution helper: the smallest offload cost (bytes, as defined
   at sparkcl_config.offload_min_bytes) at which running a task on this GPU
   beats a host path that processes `host_bytes_per_s`.  The GPU side is
   measured once per context: the fixed cost of one blocking offload
   (launch, completion, result copy back) and the streaming rate of a large
   reduce; then bytes = fixed / (1/host - 1/gpu).  UINT64_MAX if the host
   path streams at least as fast.  Needs 256 MiB of free arena the first
   time (ENOMEM otherwise). */
SPARKCL_API int sparkcl_offload_breakeven(sparkcl_ctx *ctx, double host_bytes_per_s,
                                          uint64_t *bytes);

/* ---- allocation-free ReduceCL ------------------------------------------ */
/* For callers that cannot allocate device memory when they call (tight
   serving loops, harnesses that forbid allocation): the batched ReduceCL of
   sparkcl_reduce_async(..., SPARKCL_BATCHED, ...) -- cut into the same tiles
   under ctx's tuning table and occupancy, so its results are bit-identical
   to that call's -- with every workspace it needs (task table, tile queue,
   partials, arrival tickets, queue counters, internal results) in one fixed
   array of SPARKCL_NOALLOC_SCRATCH_BYTES of device memory that the library
   holds on each GPU it runs on until the process ends, instead of blocks of
   the context's arena.  The call allocates nothing (no hipMalloc, no arena
   block, no heap memory when it succeeds); ctx supplies the device, the
   tuning table, the occupancy and the offload threshold only.
   tasks (host memory) and the inputs they name are as for sparkcl_reduce;
   results go to dev_per_task[ntasks] and *dev_total (device memory,
   caller-owned, either may be NULL; with dev_per_task set and dev_total NULL
   the RDD total is not computed) in the order of `stream`.
   Limits: at most SPARKCL_NOALLOC_MAX_TASKS tasks and, after decomposition,
   SPARKCL_NOALLOC_MAX_TILES tiles (ETOOBIG beyond); device-resident inputs
   only (EINVAL for host-input tasks); not on a stream under capture (EINVAL);
   devices 0..63.
   Every call on one GPU shares that GPU's array, which keeps the last call's
   contents; each call clears what must start at zero.  Calls that overlapped
   on one GPU would race on it, so calls are serialised: a process-wide lock,
   and before the array is rewritten a host wait until the previous
   allocation-free call's kernels (on any stream) have finished.  A call
   therefore blocks while the previous one still runs; it does not wait for
   its own kernels. */
#define SPARKCL_NOALLOC_MAX_TASKS 8192u
#define SPARKCL_NOALLOC_MAX_TILES 262144u
#define SPARKCL_NOALLOC_SCRATCH_BYTES 12190208u /* 11.6 MiB per GPU */
SPARKCL_API int sparkcl_reduce_noalloc(sparkcl_ctx *ctx, const sparkcl_task *tasks,
                                       uint32_t ntasks, sparkcl_result *dev_per_task,
                                       sparkcl_result *dev_total, void *stream);

/* Library version string. */
SPARKCL_API const char *sparkcl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPARKCL_H */
