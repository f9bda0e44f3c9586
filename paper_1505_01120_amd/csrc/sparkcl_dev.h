// Device-format descriptors shared by the host runtime and the HIP kernels of
// the SparkCL hot path.  Not part of the public ABI (include/sparkcl.h).
#pragma once

#include <stdint.h>

#include "sparkcl.h"

namespace sparkcl {

// Threads per block of the tile kernels (the default, and the only size of
// the serving, chain, map, tree and word-count kernels).  The batch executor
// and the per-partition kernel also run 512- and 1024-thread blocks, as the
// tuning table says.  The per-thread element order inside a tile, and so
// the rounding of its sum, depends on the block size, the quads in flight
// per thread and the tile size only.
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlock = 1024;
constexpr int kMaxWaves = kMaxBlock / 64;
// Loads in flight per thread in the streaming loops (float4 per input): the
// default; the tuning table picks 2, 4 or 8 per kernel.
constexpr int kUnroll = 4;

// Kernel body selector, derived on the host from (kernel id, degree, output).
enum Variant : uint32_t {
    V_POLY = 0,   // V_POLY + d: POLY of degree d, reduce only
    V_POLYW = 8,  // V_POLYW + d: POLY of degree d, reduce and write map output
    V_FMUL = 16,  // FMUL, reduce only
    V_FMULW = 17, // FMUL, reduce and write map output
    V_MC = 18,    // MC_PI hit count
    V_DECLINED = 19, // declined by selective execution: no work, status EDECLINED
    V_COUNT = 19
};

// One tile's block-combined partial result.
struct Partial {
    double sum;
    float max;
    uint32_t pad;
    uint64_t count;
    uint64_t n;
};
static_assert(sizeof(Partial) == 32, "Partial layout");

// A partition task as the kernels read it (128 B, one cache line pair).
struct TaskDev {
    uint16_t kid;
    uint16_t unroll;     // quads in flight per thread and input: 2, 4 or 8
    uint32_t ops;
    uint64_t n;
    const float *in0;
    const float *in1;
    float *out;
    uint64_t seed;
    uint32_t pid;
    uint32_t variant;
    float coef[8];
    float c;
    uint32_t tile_elems; // tile size in elements (samples for MC_PI); even
    uint32_t ntiles;     // >= 1 (an empty task has one empty tile)
    uint32_t index;      // result / sync slot of this task
    Partial *partials;   // ntiles entries
    uint64_t seq;        // serving sequence number (0 in batch launches)
    uint64_t tile_first; // serving: global index of the task's first tile
};
static_assert(sizeof(TaskDev) == 128, "TaskDev layout");

// Per-task arrival ticket of the last-block combine; self-resetting.
struct TaskSync {
    uint32_t ticket;
    uint32_t pad;
    uint64_t t_start; // min device time over the task's tiles; reset to ~0
};
static_assert(sizeof(TaskSync) == 16, "TaskSync layout");

// Persistent-executor queue state; every field returns to zero at kernel end
// so the next launch needs no clearing.
struct BatchCtl {
    uint32_t head;       // next tile to hand out
    uint32_t exited;     // blocks that have left the loop
    uint32_t rdd_ticket; // tasks finished (RDD-level combine)
    uint32_t pad;
};

struct TileRef {
    uint32_t task;
    uint32_t tile;
};

// Where a launch writes its results.
struct LaunchOut {
    TaskSync *sync;          // per task index
    BatchCtl *ctl;
    sparkcl_result *results; // per task index, contiguous
    sparkcl_result *total;   // RDD-level total, or nullptr
    uint64_t *done;          // serving: completion words (seq + 1), or nullptr
    uint32_t ntasks;         // tasks in the RDD-level combine (0: none)
    uint32_t ns_per_tick;    // device wall clock period
};

// Serving: host-visible control words of the resident executor (pinned,
// host-coherent memory).
struct ServeHost {
    uint64_t tail;  // tasks published by the host (release-stored)
    uint64_t stop;  // 1: drain published tiles and exit; 2: abort at once
    uint64_t pad[6];
};

// Serving: device-side state of the resident executor.  It persists across
// relaunches (an idle executor exits and is started again on demand).  The
// polled word, the claim counter and the dispatcher's own counter sit on
// separate 128-byte lines so polling does not contend with claims.
constexpr uint64_t kServeStopBit = 1ull << 63;  // drain published tiles, then exit
constexpr uint64_t kServeAbortBit = 1ull << 62; // exit without running more tiles
constexpr uint64_t kServeCountMask = kServeAbortBit - 1;
struct ServeDev {
    uint64_t tiles_pub; // tiles published to the workers; kServeStopBit: exit
    uint64_t pad0[15];
    uint64_t claim;     // next tile ticket handed to a worker
    uint64_t pad1[15];
    uint64_t taken;     // host-ring tasks copied into the device table
    uint64_t pad2[15];
};
static_assert(sizeof(ServeDev) == 384, "ServeDev layout");

struct ServeArgs {
    ServeHost *host;     // host-coherent control words
    const TaskDev *ring; // host-coherent descriptor ring [cap]
    ServeDev *dev;       // device control block
    TaskDev *table;      // device copy of the descriptors [cap]
    uint32_t *tilemap;   // device tile -> slot map [tile_cap]
    LaunchOut out;       // sync per slot, host results, host done words
    uint32_t cap;        // ring capacity (power of two)
    uint32_t tile_cap;   // tile map capacity (power of two)
    uint64_t idle_ticks; // executor exits after this many idle clock ticks
};

// ---- launchers (kernels.hip) ---------------------------------------------
int launch_task(const TaskDev *dtask, uint32_t ntiles, uint32_t grid,
                const LaunchOut &out, void *stream, uint32_t block = kBlock);
// mc_only: every task is a Monte-Carlo one (or declined), run by the
// executor instance that holds only the Philox body.
int launch_batch(const TaskDev *dtasks, const TileRef *tiles, uint32_t ntiles,
                 uint32_t grid, const LaunchOut &out, void *stream, uint32_t block = kBlock,
                 bool mc_only = false);
int launch_map(const TaskDev *dtask, uint64_t n, uint32_t variant,
               uint32_t grid, void *stream);
int launch_zero(void *p, uint64_t bytes, void *stream);
// Map chains: up to kMaxPost POLY stages after a task's registry map.
constexpr int kMaxPost = 4;
struct ChainDev {
    uint32_t npost;
    uint32_t deg[kMaxPost];
    float coef[kMaxPost][8];
};
// One persistent-executor launch over a batched tile queue whose tasks all
// run the chain `chain` after their own map; `unroll` float4 loads (4 or 8)
// in flight per thread and input.
int launch_chain(const TaskDev *dtasks, const TileRef *tiles, uint32_t ntiles,
                 const ChainDev *chain, uint32_t grid, const LaunchOut &out, uint32_t unroll,
                 void *stream);
// Array-valued ReduceCL, one pass: reduces `count` leaves of `len` floats
// (from the device pointer table `ptrs`, or, when ptrs is null, the rows
// base + i * stride) in chunks of `chunk` leaves; chunk c's tree goes to
// out + c * len.
struct TreeArgs {
    const float *const *ptrs;
    const float *base;
    uint64_t stride;
    float *out;
    uint64_t len;
    uint32_t count;
    uint32_t chunk;
    uint32_t cpt; // float4 columns per thread: 1 (8-leaf groups), or 2 / 4
                  // (leaf pairs, chunks of at most kTreeWideChunk leaves)
    uint32_t threads; // block threads of the leaf-pair kernel: kBlock, or
                      // kTreeWideBig with 4 columns per thread
};
constexpr uint32_t kTreeWideChunk = 64;
constexpr uint32_t kTreeWideBig = 512;
int launch_tree(const TreeArgs &a, uint32_t combiner, bool vec4, void *stream);
// WordCount: text of n bytes counted into the global open-addressing table
// keys/counts of mask + 1 slots (a power of two, cleared beforehand); ctl[0]
// words, ctl[1] count of the key 0, ctl[2] table-full flag, ctl[3] distinct
// keys written by the compaction.
// Words that miss a block's LDS table are appended to the block's spill
// region of their key's partition (the top kWcPartBits bits of the key),
// spill_cap keys per region, counts in spill_cnt, instead of being added to
// the global table one atomic at a time; the merge kernel then counts each
// partition's spilled keys in LDS and adds each distinct key to the table
// once per merge block.  spill_cap 0: no spill regions (every miss goes to
// the table directly).
constexpr uint32_t kWcPartBits = 8;
struct WcArgs {
    const uint8_t *text;
    uint64_t n;
    uint64_t *keys;
    uint64_t *counts;
    uint64_t mask;       // table slots - 1 (a power of two minus one)
    uint64_t *ctl;       // words, zero-key count, table full, distinct keys
    uint32_t spill_cap;  // keys per spill region (0: no spill regions)
    uint32_t pad;
    uint64_t *spill;     // [scan block][partition][spill_cap]
    uint32_t *spill_cnt; // [scan block][partition] keys written
};
int launch_wordcount(const WcArgs &a, uint32_t grid, void *stream);
// Merge of the spill regions of `scan_grid` scan blocks into the table, with
// `per_part` blocks per partition.
int launch_wc_merge(const WcArgs &a, uint32_t scan_grid, uint32_t per_part, void *stream);
int launch_wc_compact(const WcArgs &a, uint64_t *keys, uint64_t *counts, uint64_t cap,
                      uint32_t grid, void *stream);
int wordcount_blocks_per_cu(int *out);
// WordCount's words: for each of nkeys distinct keys, the byte offset of the
// first word with that key (UINT64_MAX if none), through a lookup table of
// mask + 1 slots (tkeys cleared to 0 and ctl[0..1] to 0 beforehand).  ctl[0]:
// index + 1 of the key 0; ctl[1]: set when a key repeats.
struct WlArgs {
    const uint8_t *text;
    uint64_t n;
    const uint64_t *keys;
    uint64_t nkeys;
    uint64_t *offsets;
    uint64_t *tkeys;     // lookup table keys (0: empty)
    uint32_t *tidx;      // the index of each table key in keys
    uint64_t mask;       // table slots - 1 (a power of two minus one)
    uint64_t *ctl;
};
int launch_wordcount_locate(const WlArgs &l, uint32_t scan_grid, void *stream);
// Resident serving executor: block 0 dispatches, the rest run tiles.  Each
// launch first discards tickets left unpublished by the previous launch.
int launch_serve(const ServeArgs &a, uint32_t workers, void *stream);
int launch_fill_pattern(float *p, uint64_t n, uint32_t salt, void *stream);
// Blocks of the batch executor (and of its Monte-Carlo-only instance) that
// fit on one CU at once.
int batch_blocks_per_cu(int *out);
int batch_mc_blocks_per_cu(int *out);
int chain_blocks_per_cu(int *out);

} // namespace sparkcl
