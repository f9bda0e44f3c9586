"""Run the library's autotuner on GPU 0 and write the tuning cache.

The autotuner (sparkcl_autotune) times, on synthetic device data, each
registry kernel's blocks per CU with its tile, its block size and loads in
flight, then candidate tile sizes for every execution mode, kernel and log2(n)
bucket, then the tiles, occupancy and block size for mixed batches of many
tasks, and stores the table in a JSON file keyed by the device's gfx arch.  Contexts load that file by default
(paper_1505_01120_amd/tuning.json), so one machine always cuts a task into the
same tiles and results stay run-to-run identical.

Usage: python -m paper_1505_01120_amd.autotune [--lo 10] [--hi 24] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import sparkcl as sc


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--lo", type=int, default=10, help="smallest log2(n) bucket")
    ap.add_argument("--hi", type=int, default=24, help="largest log2(n) bucket")
    ap.add_argument("--out", default=sc.TUNING_PATH)
    args = ap.parse_args(argv)
    t0 = time.time()
    # start from the built-in defaults, not from an existing cache
    with sc.Context(device=0, arena_bytes=3 << 30, tune_cache=None) as ctx:
        ctx.autotune(args.lo, args.hi, args.out)
        t = ctx.get_tuning()
    names = ["per_launch", "batched", "serve"]
    kern = ["poly", "fmul", "mc_pi"]
    summary = {"blocks_per_cu": list(t.blocks_per_cu),
               "blocks_per_cu_many": t.blocks_per_cu_many,
               "tile_many": list(t.tile_many),
               "many_tiles_per_cu": list(t.many_tiles_per_cu),
               "blocks_per_cu_mc_only": t.blocks_per_cu_mc_only,
               "block": list(t.block), "block_many": t.block_many,
               "unroll": list(t.unroll),
               "tiles": {m: {k: list(t.tile[i][j][args.lo:args.hi + 1])
                             for j, k in enumerate(kern)} for i, m in enumerate(names[:2])}}
    print(json.dumps(summary), flush=True)
    print(f"wrote {args.out} in {time.time() - t0:.1f} s", file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
