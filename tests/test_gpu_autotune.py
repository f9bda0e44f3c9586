"""The autotuner (sparkcl_autotune) on the GPU, over a narrow range of size
buckets: it leaves a table whose every entry the library accepts, writes it
to the JSON cache, a new context reads back the identical table from that
cache (the tuned choice is fixed per architecture key, not re-drawn per run),
and reductions under the tuned table still match the oracle."""
import ctypes
import math

import pytest

import datagen
from gpu_helpers import DevParts, check_result, check_total, oracle_result
import paper_1505_01120_amd as sc

pytestmark = pytest.mark.gpu

MIN_TILE, MAX_TILE = 1 << 10, 1 << 22


def entries(t: sc.Tuning):
    return (list(t.blocks_per_cu) + [t.blocks_per_cu_many] + list(t.tile_many) +
            list(t.block) + [t.block_many] + list(t.unroll) + list(t.many_tiles_per_cu) +
            [t.blocks_per_cu_mc_only] +
            [t.tile[m][k][b] for m in range(sc.TUNE_MODES) for k in range(3)
             for b in range(sc.TUNE_BUCKETS)])


def test_autotune_table_cache_and_parity(tmp_path):
    path = str(tmp_path / "tuning.json")
    c = sc.Context(device=0, arena_bytes=3 << 30, tune_cache=None)
    try:
        c.autotune(12, 13, path)
        tuned = c.get_tuning()
    finally:
        c.destroy()

    for b in list(tuned.blocks_per_cu) + [tuned.blocks_per_cu_many, tuned.blocks_per_cu_mc_only]:
        assert 1 <= b <= 16, b
    for b in list(tuned.block) + [tuned.block_many]:
        assert b in (256, 512, 1024), b
    for u in tuned.unroll:
        assert u in (2, 4, 8), u
    assert tuned.unroll[2] == 4  # the Monte-Carlo kernel has no streaming loop
    for q in tuned.many_tiles_per_cu:
        assert q in (0, 4, 8, 12, 16, 24, 32, 48, 64, 128), q
    for v in tuned.tile_many:
        assert v == 0 or (MIN_TILE <= v <= MAX_TILE and v & (v - 1) == 0), v
    for m in range(sc.TUNE_MODES):
        for k in range(3):
            for b in range(sc.TUNE_BUCKETS):
                v = tuned.tile[m][k][b]
                assert MIN_TILE <= v <= MAX_TILE and v & (v - 1) == 0, (m, k, b, v)

    c2 = sc.Context(device=0, arena_bytes=1 << 30, tune_cache=path)
    try:
        loaded = c2.get_tuning()
        assert ctypes.string_at(ctypes.addressof(loaded), ctypes.sizeof(loaded)) == \
            ctypes.string_at(ctypes.addressof(tuned), ctypes.sizeof(tuned)), \
            [(i, a, b) for i, (a, b) in enumerate(zip(entries(loaded), entries(tuned))) if a != b]
        parts = [datagen.make_part(k, n, i) for i, (k, n) in enumerate(
            [(datagen.POLY, 5000), (datagen.FMUL, 8192 + 3), (datagen.MC_PI, 70_000),
             (datagen.FMUL, 1 << 18)])]
        d = DevParts(parts, 1, 2)
        for mode in (sc.PER_LAUNCH, sc.BATCHED, sc.GRAPH):
            per, _ = c2.reduce(d.tasks, mode)
            for p, g in zip(parts, per):
                check_result(g, oracle_result(p), p.kid, p.ops, f"mode {mode} kid {p.kid} n {p.n}")
        # a mixed batch of many tasks: the tuned mixed-batch tiles, occupancy
        # and block size
        sizes = datagen.lognormal_sizes(700, 11, 3, 8192, math.log(4.0), 16, 300_000)
        kids = datagen.uniform_kernel_ids(700, 11, 4)
        parts = [datagen.make_part(int(k), int(n), i) for i, (n, k) in enumerate(zip(sizes, kids))]
        d = DevParts(parts, 3, 1)
        want = [oracle_result(p) for p in parts]
        for mode in (sc.BATCHED, sc.GRAPH):
            per, tot = c2.reduce(d.tasks, mode)
            for p, g, o in zip(parts, per, want):
                check_result(g, o, p.kid, p.ops, f"mixed mode {mode} kid {p.kid} n {p.n}")
            check_total(tot, want, datagen.SUM | datagen.MAX | datagen.COUNT)
    finally:
        c2.destroy()
