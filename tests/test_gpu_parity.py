"""GPU parity: the HIP path through the C ABI against the oracle, element by
element on the same seeded inputs (MapCL, MapCLPartition, ReduceCL; paper
sec. 3.1.3).  Sizes span several tiles with ragged tails; the full-size
workloads (the 64 x 2^22 RDD, 256 x 2^24 Monte-Carlo samples, the 4096-task
uneven batch) are checked partition by partition, with the RDD totals.
"""
import math

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, check_total, dev, oracle_result

pytestmark = pytest.mark.gpu

MODES = [sc.PER_LAUNCH, sc.BATCHED, sc.GRAPH]
EDGE_N = [0, 1, 3, 4, 5, 63, 64, 65, 255, 257, 1023, 1025, 4095, 4097, 65535,
          65537, 131073, 1 << 20, (1 << 20) + 3]


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=2 << 30)
    yield c
    c.destroy()


def run_and_check(ctx, parts, mode, xoff=0, yoff=0):
    d = DevParts(parts, xoff, yoff)
    per, tot = ctx.reduce(d.tasks, mode)
    want = [oracle_result(p) for p in parts]
    for p, g, o in zip(parts, per, want):
        check_result(g, o, p.kid, p.ops, f"kid={p.kid} n={p.n} pid={p.pid} mode={mode}")
    ops = 0
    for p in parts:
        ops |= p.ops
    check_total(tot, want, ops)
    return per, tot


@pytest.mark.parametrize("mode", MODES)
def test_single_partition_poly_sum(ctx, mode):
    # 2^20 floats U[-1,1) from seed 0, y = 0.5x^2 - 1.25x + 3, SUM
    run_and_check(ctx, datagen.single_partition(), mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kid", [datagen.POLY, datagen.FMUL])
def test_edge_sizes(ctx, mode, kid):
    parts = [datagen.make_part(kid, n, pid) for pid, n in enumerate(EDGE_N)]
    run_and_check(ctx, parts, mode)


@pytest.mark.parametrize("mode", MODES)
def test_mc_counts_bit_exact(ctx, mode):
    sizes = [0, 1, 2, 3, 4, 5, 1023, 4097, 65536, 65537, 1 << 20, (1 << 20) + 1]
    parts = [datagen.make_part(datagen.MC_PI, n, pid, with_data=False)
             for pid, n in enumerate(sizes)]
    parts.append(datagen.Part(kid=datagen.MC_PI, ops=datagen.COUNT, n=99_999, pid=7,
                              seed=0xDEADBEEF12345678))
    run_and_check(ctx, parts, mode)


@pytest.mark.parametrize("mode", MODES)
def test_map_partition_mc(ctx, mode):
    parts = [datagen.make_part(datagen.MC_PI, 300_001 + p, p, with_data=False)
             for p in range(6)]
    d = DevParts(parts)
    res = ctx.map_partition(d.tasks, mode)
    for p, g in zip(parts, res):
        check_result(g, oracle_result(p), p.kid, p.ops, f"pid={p.pid}")


@pytest.mark.parametrize("mode", MODES)
def test_ops_subsets(ctx, mode):
    parts = [datagen.make_part(datagen.FMUL, 70_001, 0, ops=datagen.SUM),
             datagen.make_part(datagen.FMUL, 70_002, 1, ops=datagen.MAX),
             datagen.make_part(datagen.POLY, 70_003, 2, ops=datagen.MAX),
             datagen.make_part(datagen.POLY, 70_004, 3, ops=datagen.SUM | datagen.MAX)]
    run_and_check(ctx, parts, mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("xoff,yoff", [(1, 1), (2, 2), (3, 3), (1, 2), (0, 3)])
def test_unaligned_inputs(ctx, mode, xoff, yoff):
    # float4 quads after a scalar head up to x's first 16-byte boundary; y
    # is read with the same quad indices at its own (4-byte) alignment
    parts = [datagen.make_part(datagen.FMUL, n, pid) for pid, n in
             enumerate([5, 1000, 65537, 300_000])]
    parts += [datagen.make_part(datagen.POLY, 65539, 9)]
    run_and_check(ctx, parts, mode, xoff, yoff)


@pytest.mark.parametrize("degree", range(8))
def test_poly_degrees(ctx, degree):
    coef = tuple(float(np.float32(0.5 - 0.125 * k)) for k in range(degree + 1))
    x = datagen.fill(40_001, 0, degree, 1, datagen.U_PM1)
    p = datagen.Part(kid=datagen.POLY, ops=datagen.SUM | datagen.MAX, n=x.size,
                     pid=degree, x=x, coef=coef)
    run_and_check(ctx, [p], sc.BATCHED)


@pytest.mark.parametrize("kid", [datagen.POLY, datagen.FMUL])
@pytest.mark.parametrize("xoff,ooff", [(0, 0), (1, 1), (1, 0), (3, 2)])
def test_map_materialised_bit_exact(ctx, kid, xoff, ooff):
    n = 100_003
    p = datagen.make_part(kid, n, 5)
    x, y = dev(p.x, xoff), dev(p.y, xoff)
    buf = torch.full((n + 8,), float("nan"), dtype=torch.float32, device="cuda")
    out = buf[ooff:ooff + n]
    ctx.map([sc.task(kid, n, x, y, out, coef=p.coef, c=p.c)])
    torch.cuda.synchronize()
    want = oracle.poly_map(p.x, p.coef) if kid == datagen.POLY else oracle.fmul_map(p.x, p.y)
    got = out.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # nothing written outside [0, n)
    assert torch.isnan(buf[:ooff]).all() and torch.isnan(buf[ooff + n:]).all()


@pytest.mark.parametrize("mode", MODES)
def test_reduce_with_materialised_output(ctx, mode):
    parts = [datagen.make_part(datagen.FMUL, 123_457, 0),
             datagen.make_part(datagen.POLY, 65_541, 1)]
    d = DevParts(parts, out=True)
    per, _ = ctx.reduce(d.tasks, mode)
    torch.cuda.synchronize()
    for p, g, o in zip(parts, per, d.outs):
        check_result(g, oracle_result(p), p.kid, p.ops, f"kid={p.kid}")
        want = oracle.poly_map(p.x, p.coef) if p.kid == datagen.POLY else \
            oracle.fmul_map(p.x, p.y)
        assert np.array_equal(o.cpu().numpy().view(np.uint32), want.view(np.uint32))


# Sizes around the chunk-interleaved tile layout (chunks of 4096 elements
# dealt round-robin to a task's tiles): fewer chunks than tiles, a partial
# last chunk owned by a tile other than 0, ragged tails and unaligned heads.
FORCED_N = [1, 4095, 4096, 4097, 4099, 8191, 3 * 4096 + 5, 5 * 4096 + 1030,
            17 * 4096 + 3, 100_003, 262_147]


@pytest.fixture
def forced_tiles(ctx):
    """Set every tile size of every mode to one value for the test's duration."""
    saved = ctx.get_tuning()

    def force(log2: int):
        t = sc.Tuning.from_buffer_copy(saved)
        for m in range(len(t.tile)):
            for k in range(len(t.tile[m])):
                for b in range(len(t.tile[m][k])):
                    t.tile[m][k][b] = 1 << log2
        ctx.set_tuning(t)

    yield force
    ctx.set_tuning(saved)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("tile_log2", [10, 12, 13, 16])
@pytest.mark.parametrize("off", [0, 1, 3])
def test_forced_tile_sizes(ctx, forced_tiles, mode, tile_log2, off):
    forced_tiles(tile_log2)
    parts = [datagen.make_part(kid, n, 8 * i + kid)
             for i, n in enumerate(FORCED_N) for kid in (datagen.POLY, datagen.FMUL)]
    d = DevParts(parts, off, off, out=True)
    per, tot = ctx.reduce(d.tasks, mode)
    torch.cuda.synchronize()
    want = [oracle_result(p) for p in parts]
    for p, g, o, buf in zip(parts, per, want, d.outs):
        where = f"kid={p.kid} n={p.n} T=2^{tile_log2} off={off} mode={mode}"
        check_result(g, o, p.kid, p.ops, where)
        m = oracle.poly_map(p.x, p.coef) if p.kid == datagen.POLY else \
            oracle.fmul_map(p.x, p.y)
        assert np.array_equal(buf.cpu().numpy().view(np.uint32), m.view(np.uint32)), where
    ops = 0
    for p in parts:
        ops |= p.ops
    check_total(tot, want, ops)


SHAPES = [(256, 2), (256, 8), (512, 4), (512, 8), (1024, 2), (1024, 4)]


@pytest.mark.parametrize("block,unroll", SHAPES)
@pytest.mark.parametrize("off", [0, 3])
def test_forced_block_and_unroll(ctx, block, unroll, off):
    # every kernel's executor block size and streaming loads in flight forced
    # to one shape (sparkcl_tuning.block, .unroll, .block_many), with small
    # tiles so that each task spans many tiles and takes the interleaved,
    # contiguous and ragged paths; per-launch, batched and graph, single-kernel
    # and mixed batches, materialised outputs, and the RDD total
    saved = ctx.get_tuning()
    t = sc.Tuning.from_buffer_copy(saved)
    for k in range(3):
        t.block[k] = block
        t.unroll[k] = unroll
        for m in range(len(t.tile)):
            for b in range(len(t.tile[m][k])):
                t.tile[m][k][b] = min(t.tile[m][k][b], 1 << 14)
    t.block_many = block
    ctx.set_tuning(t)
    try:
        sizes = [1, 4095, 4097, 3 * 16384 + 5, 100_003, 262_147, 1 << 20]
        mixed = [datagen.make_part(kid, n, 8 * i + kid, with_data=kid != datagen.MC_PI)
                 for i, n in enumerate(sizes)
                 for kid in (datagen.POLY, datagen.FMUL, datagen.MC_PI)]
        single = [p for p in mixed if p.kid == datagen.FMUL]
        for parts in (mixed, single):
            d = DevParts(parts, off, off, out=True)
            want = [oracle_result(p) for p in parts]
            ops = 0
            for p in parts:
                ops |= p.ops
            for mode in MODES:
                per, tot = ctx.reduce(d.tasks, mode)
                torch.cuda.synchronize()
                shape = ctx.last_launch_shape()
                assert shape["mode"] == mode and shape["ntasks"] == len(parts), shape
                if mode == sc.PER_LAUNCH:
                    assert shape["grid"] == 0 and shape["tile_table"] == 0, shape
                    assert shape["block"] == (0 if parts is mixed else block), shape
                else:
                    assert shape["block"] == block and 0 < shape["grid"] <= shape["ntiles"], shape
                for p, g, o, buf in zip(parts, per, want, d.outs):
                    where = f"kid={p.kid} n={p.n} B={block} U={unroll} off={off} mode={mode}"
                    check_result(g, o, p.kid, p.ops, where)
                    if buf is not None:
                        m = oracle.poly_map(p.x, p.coef) if p.kid == datagen.POLY else \
                            oracle.fmul_map(p.x, p.y)
                        assert np.array_equal(buf.cpu().numpy().view(np.uint32),
                                              m.view(np.uint32)), where
                check_total(tot, want, ops)
    finally:
        ctx.set_tuning(saved)


def test_block_and_unroll_refused_out_of_range(ctx):
    saved = ctx.get_tuning()
    for field, value in (("block_many", 128), ("block_many", 768)):
        t = sc.Tuning.from_buffer_copy(saved)
        setattr(t, field, value)
        with pytest.raises(sc.SparkclError):
            ctx.set_tuning(t)
    t = sc.Tuning.from_buffer_copy(saved)
    t.unroll[1] = 3
    with pytest.raises(sc.SparkclError):
        ctx.set_tuning(t)
    t = sc.Tuning.from_buffer_copy(saved)
    t.block[0] = 2048
    with pytest.raises(sc.SparkclError):
        ctx.set_tuning(t)
    assert bytes(ctx.get_tuning()) == bytes(saved)


@pytest.mark.parametrize("mode", MODES)
def test_repeat_is_bit_identical_and_async_matches(ctx, mode):
    parts = [datagen.make_part(k, 200_000 + 17 * i, i)
             for i, k in enumerate([1, 2, 3, 2, 1, 3, 2])]
    d = DevParts(parts)
    first, tot1 = ctx.reduce(d.tasks, mode)
    for _ in range(3):  # cached plan, relaunched
        again, tot2 = ctx.reduce(d.tasks, mode)
        assert [r.as_dict() | {"t_start_ns": 0, "t_done_ns": 0} for r in again] == \
               [r.as_dict() | {"t_start_ns": 0, "t_done_ns": 0} for r in first]
        assert (tot2.sum, tot2.max, tot2.count, tot2.n) == (tot1.sum, tot1.max,
                                                            tot1.count, tot1.n)
    dres = torch.zeros(64 * len(parts), dtype=torch.uint8, device="cuda")
    dtot = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        ctx.reduce_async(d.tasks, mode, dres, dtot)
    torch.cuda.synchronize()
    raw = dres.cpu().numpy()
    for i, r in enumerate(first):
        g = sc.Result.from_buffer_copy(raw[64 * i:64 * (i + 1)].tobytes())
        assert (g.sum, g.max, g.count, g.n, g.status) == (r.sum, r.max, r.count, r.n, 0)
    gt = sc.Result.from_buffer_copy(dtot.cpu().numpy().tobytes())
    assert (gt.sum, gt.count, gt.n) == (tot1.sum, tot1.count, tot1.n)
    assert ctx.last_kernel_ms() > 0


def test_errors(ctx):
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce([sc.task(9, 16, x)], sc.BATCHED)
    assert e.value.code == sc.ENOKERNEL
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce([sc.task(sc.POLY, 16, x, ops=sc.COUNT)], sc.BATCHED)
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce([sc.task(sc.FMUL, 16, x, None)], sc.PER_LAUNCH)
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.map([sc.task(sc.MC_PI, 16)])
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.map_partition([sc.task(sc.POLY, 16, x, coef=(1.0,))])
    assert e.value.code == sc.EINVAL
    bad = sc.task(sc.POLY, 16, x, coef=(1.0,))
    bad.degree = 8
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce([bad], sc.BATCHED)
    assert e.value.code == sc.EINVAL
    # the context still works after errors
    per, tot = ctx.reduce([sc.task(sc.POLY, 16, x, coef=(2.0,))], sc.BATCHED)
    assert per[0].sum == 32.0 and tot.sum == 32.0


def test_fmul_rdd_full_size(ctx):
    # 64 partitions x 2^22 pairs (x~N(0,1), y~U[0,2)); every partition checked
    # in each mode, then in the benchmark's two other launch configurations
    # of the same RDD: every y one element off x's 16-byte alignment
    # (batched), and the partitions streamed from pinned host memory
    parts = datagen.fmul_rdd()
    want = [oracle_result(p) for p in parts]

    def check_all(per, tot, where):
        for p, g, o in zip(parts, per, want):
            check_result(g, o, p.kid, p.ops, f"pid={p.pid} {where}")
        check_total(tot, want, datagen.SUM | datagen.MAX)

    d = DevParts(parts)
    for mode in MODES:
        per, tot = ctx.reduce(d.tasks, mode)
        check_all(per, tot, f"mode={mode}")
    del d
    d = DevParts(parts, 0, 1)
    per, tot = ctx.reduce(d.tasks, sc.BATCHED)
    check_all(per, tot, "y one element off")
    del d
    keep, htasks = [], []
    for p in parts:
        hx = torch.from_numpy(p.x).pin_memory()
        hy = torch.from_numpy(p.y).pin_memory()
        keep += [hx, hy]
        htasks.append(sc.task(p.kid, p.n, hx, hy, ops=p.ops, c=p.c, host=True))
    per, tot = ctx.reduce(htasks, sc.BATCHED)
    check_all(per, tot, "host input")


def oracle_parallel(fn, items, threads: int = 16):
    """Runs the single-threaded oracle on independent partitions side by side
    (each call releases the GIL inside the C oracle)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


def test_monte_carlo_full_size(ctx):
    # 256 partitions x 2^24 samples in the batched and graph launches: every
    # partition's count bit-exact against the oracle (run partition-parallel
    # on the host), every count within 5 sigma of pi/4, and the RDD total
    # against the oracle's combine of the partition results
    parts = datagen.monte_carlo()
    n = 1 << 24
    want = oracle_parallel(oracle_result, parts)
    d = DevParts(parts)
    p4 = math.pi / 4
    sigma = math.sqrt(p4 * (1 - p4) / n)
    for mode in (sc.BATCHED, sc.GRAPH):
        per, tot = ctx.reduce(d.tasks, mode)
        for p, g, o in zip(parts, per, want):
            check_result(g, o, p.kid, p.ops, f"pid={p.pid} mode={mode}")
            assert abs(g.count / n - p4) < 5 * sigma
        check_total(tot, want, datagen.COUNT)
        assert tot.n == 256 * n


def test_beyond_32_bit_element_counts(ctx):
    # One partition of 2^32 + 7 floats (16 GiB): element indices past 32 bits
    # in the batched, graph and per-launch paths and in the materialised map.
    # x is 1 except at a few marked positions, so the sum has a closed form
    # that FP64 holds exactly (integers and halves below 2^53).
    n = (1 << 32) + 7
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    marks = [0, (1 << 31) + 1, (1 << 32) - 1, 1 << 32, n - 1]
    vals = [2.0, 3.0, 0.5, 4.0, 8.0]
    for i, v in zip(marks, vals):
        x[i] = v
    want = float(n - len(marks)) + sum(vals)
    t = sc.task(sc.POLY, n, x, coef=(0.0, 1.0))  # y = x
    for mode in MODES:
        per, tot = ctx.reduce([t], mode)
        assert (per[0].n, per[0].sum, per[0].max, per[0].status) == (n, want, 8.0, 0), mode
        assert (tot.n, tot.sum) == (n, want)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.map([sc.task(sc.POLY, n, x, out=out, coef=(0.5, 2.0))])  # y = 0.5 + 2x, exact
    torch.cuda.synchronize()
    for i, v in zip(marks, vals):
        assert out[i].item() == 0.5 + 2.0 * v, i
    for i in (1, 12345, (1 << 32) + 3):
        assert out[i].item() == 2.5, i
    del x, out
    torch.cuda.empty_cache()


def share_tile(total: float, cus: int, q: int) -> int:
    """The mixed-batch tile a work share gives: total / (CUs x q) rounded to
    the nearest power of two (log2 rounded half to even), clamped to
    [2^10, 2^22]."""
    if q == 0 or total == 0:
        return 0
    e = int(np.rint(math.log2(max(total / (cus * q), 1.0))))
    return 1 << min(22, max(10, e))


@pytest.mark.parametrize("many,share", [((4096, 8192, 2048), (0, 0)),
                                        ((1 << 16, 1 << 16, 1 << 15), (0, 0)),
                                        ((0, 1024, 0), (0, 0)),
                                        ((0, 0, 0), (16, 8)),
                                        ((0, 4096, 0), (64, 2))])
def test_mixed_batch_tile_sizes(ctx, many, share):
    # 600 tasks spanning many size buckets take the mixed-batch tile sizes in
    # batched modes: given per kernel (sparkcl_tuning.tile_many), else derived
    # from the batch's totals and a number of tiles per CU
    # (many_tiles_per_cu), else the per-bucket table
    sizes = datagen.lognormal_sizes(600, 9, 3, 8192, math.log(4.0), 16, 300_000)
    kids = datagen.uniform_kernel_ids(600, 9, 4)
    parts = [datagen.make_part(int(k), int(n), i) for i, (n, k) in enumerate(zip(sizes, kids))]
    saved = ctx.get_tuning()
    t = sc.Tuning.from_buffer_copy(saved)
    for k in range(3):
        t.tile_many[k] = many[k]
    t.many_tiles_per_cu[0], t.many_tiles_per_cu[1] = share
    ctx.set_tuning(t)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    # streaming work in input bytes (4 per POLY element, 8 per FMUL element)
    stream = sum(p.n * (8 if p.kid == datagen.FMUL else 4) for p in parts
                 if p.kid != datagen.MC_PI)
    mc = sum(p.n for p in parts if p.kid == datagen.MC_PI)
    want = [many[0] or share_tile(stream / 4, cus, share[0]),
            many[1] or share_tile(stream / 8, cus, share[0]),
            many[2] or share_tile(mc, cus, share[1])]
    try:
        for mode in (sc.BATCHED, sc.GRAPH):
            run_and_check(ctx, parts, mode)
            shape = ctx.last_launch_shape()
            if many[0] == 1 << 16:
                # 2^16 tiles leave the executor's blocks under two tiles each:
                # the batch is cut with the per-launch table instead
                assert shape["tile_table"] == 0 and shape["mixed"] == 0, shape
                assert shape["mixed_tile"] == [0, 0, 0], shape
            else:
                assert shape["mixed"] == 1 and shape["tile_table"] == 1, shape
                assert shape["mixed_tile"] == want, (shape, want)
    finally:
        ctx.set_tuning(saved)


def test_uneven_batch_reduced(ctx):
    # log-normal sizes (median 4K, clipped 16..256K) with mixed kernels
    sizes = datagen.lognormal_sizes(300, 5, 3, 4096, math.log(4.0), 16, 262144)
    kids = datagen.uniform_kernel_ids(300, 5, 4)
    parts = [datagen.make_part(int(k), int(n), i) for i, (n, k) in enumerate(zip(sizes, kids))]
    for mode in MODES:
        run_and_check(ctx, parts, mode)


def test_uneven_batch_full_size(ctx):
    # The benchmark's 4096-partition log-normal batch (mixed kernels; one
    # device pool per input, each partition's slice 256-byte aligned) at full
    # size, in its batched launch (the mixed-batch tiles and occupancy) and
    # replayed from its graph: every partition and the RDD total against the
    # oracle (run partition-parallel on the host).
    sizes, kids = datagen.uneven_sizes()
    parts = [datagen.make_part(int(k), int(n), p) for p, (n, k) in enumerate(zip(sizes, kids))]

    def up(v):
        return (v + 63) // 64 * 64
    nx = sum(up(p.n) for p in parts if p.kid != datagen.MC_PI)
    ny = sum(up(p.n) for p in parts if p.kid == datagen.FMUL)
    x = torch.empty(nx, dtype=torch.float32, device="cuda")
    y = torch.empty(max(ny, 1), dtype=torch.float32, device="cuda")
    tasks, ox, oy = [], 0, 0
    for p in parts:
        if p.kid == datagen.MC_PI:
            tasks.append(sc.task(p.kid, p.n, pid=p.pid, seed=p.seed))
            continue
        xs = x[ox:ox + p.n]
        xs.copy_(torch.from_numpy(p.x))
        ox += up(p.n)
        ys = None
        if p.kid == datagen.FMUL:
            ys = y[oy:oy + p.n]
            ys.copy_(torch.from_numpy(p.y))
            oy += up(p.n)
        tasks.append(sc.task(p.kid, p.n, xs, ys, ops=p.ops, coef=p.coef, c=p.c))
    want = oracle_parallel(oracle_result, parts)
    ops = datagen.SUM | datagen.MAX | datagen.COUNT
    for mode in (sc.BATCHED, sc.GRAPH):
        per, tot = ctx.reduce(tasks, mode)
        for p, g, o in zip(parts, per, want):
            check_result(g, o, p.kid, p.ops, f"pid={p.pid} kid={p.kid} n={p.n} mode={mode}")
        check_total(tot, want, ops)
        assert tot.n == int(sizes.sum())


def test_launch_shape_follows_the_occupancy_rules():
    # A batch of Monte-Carlo tasks alone runs the executor instance of its
    # own at blocks_per_cu_mc_only; a batch that mixes kernels takes the
    # largest of its kernels' blocks_per_cu.  Counts against the oracle in
    # both.  Before any reduce-kind call the shape query says EAGAIN.
    c = sc.Context(device=0, arena_bytes=1 << 30)
    try:
        with pytest.raises(sc.SparkclError) as e:
            c.last_launch_shape()
        assert e.value.code == sc.EAGAIN
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        t = c.get_tuning()
        t.blocks_per_cu[0], t.blocks_per_cu[1], t.blocks_per_cu[2] = 2, 1, 3
        t.blocks_per_cu_mc_only = 5
        t.blocks_per_cu_many = 1
        for m in range(len(t.tile)):
            t.tile[m][2][20] = 1 << 12   # 256 tiles per 2^20-sample task
            t.tile[m][0][20] = 1 << 14
        c.set_tuning(t)
        mc = [datagen.make_part(datagen.MC_PI, 1 << 20, pid, with_data=False)
              for pid in range(16)]
        for mode in (sc.BATCHED, sc.GRAPH):
            per, _ = c.reduce(DevParts(mc).tasks, mode)
            for p, g in zip(mc, per):
                check_result(g, oracle_result(p), p.kid, p.ops, f"mc pid={p.pid} mode={mode}")
            shape = c.last_launch_shape()
            assert shape["grid"] == 5 * cus and shape["ntiles"] == 16 * 256, shape
        mixed = mc[:8] + [datagen.make_part(datagen.POLY, 1 << 20, 100 + i) for i in range(8)]
        d = DevParts(mixed)
        per, _ = c.reduce(d.tasks, sc.BATCHED)
        for p, g in zip(mixed, per):
            check_result(g, oracle_result(p), p.kid, p.ops, f"mixed kid={p.kid} pid={p.pid}")
        shape = c.last_launch_shape()
        assert shape["grid"] == 3 * cus, shape
    finally:
        c.destroy()
