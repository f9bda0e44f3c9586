// Tile-size table of the SparkCL hot path: per execution mode, kernel and
// log2(n) bucket, the number of elements one block handles per tile.  The
// decomposition of a task is a pure function of (mode, kernel id, n) under a
// given table, which is what makes results schedule-independent.
// Pure host logic: defaults, validation, and the JSON cache format.
#pragma once

#include <cstdint>
#include <map>
#include <string>

#include "sparkcl.h"

namespace sparkcl {

enum TuneMode { TM_PER_LAUNCH = 0, TM_BATCHED = 1, TM_SERVE = 2 };

constexpr uint32_t kMinTileLog2 = 10;
constexpr uint32_t kMaxTileLog2 = 22;

inline uint32_t size_bucket(uint64_t n)
{
    uint32_t b = 0;
    while (b < SPARKCL_TUNE_BUCKETS - 1 && (n >> (b + 1)) != 0)
        ++b;
    return b;
}

void tuning_defaults(sparkcl_tuning *t);
// SPARKCL_OK or SPARKCL_EINVAL (with a reason in *why).
int tuning_validate(const sparkcl_tuning *t, std::string *why);
uint32_t tile_for(const sparkcl_tuning &t, int mode, uint32_t kid, uint64_t n);

// JSON cache: { "<gfx arch>": { "blocks_per_cu": [P, F, M], "blocks_per_cu_many":
// N, "blocks_per_cu_mc_only": N, "tile_many": [P, F, M], "block": [P, F, M], "block_many": N, "unroll":
// [P, F, M], "many_tiles_per_cu": [S, M], "tile": { "<mode>": { "<kernel>":
// [32 tile sizes] } } }, ... }
// with modes per_launch, batched, serve and kernels poly, fmul, mc_pi; keys
// left out keep their defaults.
bool tuning_parse_json(const std::string &text,
                       std::map<std::string, sparkcl_tuning> *out,
                       std::string *err);
std::string tuning_to_json(const std::map<std::string, sparkcl_tuning> &all);
bool tuning_load_file(const std::string &path, const std::string &arch,
                      sparkcl_tuning *out, std::string *err);
bool tuning_save_file(const std::string &path, const std::string &arch,
                      const sparkcl_tuning &t, std::string *err);

} // namespace sparkcl
