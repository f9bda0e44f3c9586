"""Selective execution (sec. 3.1.1: a kernel may decline accelerated
execution, and mapReturnValue then calls an alternative function): tasks
whose offload cost is below the context's threshold are declined -- not run,
status SPARKCL_EDECLINED, nothing added to the RDD total -- and the rest
match the oracle."""
import time

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, oracle_result

pytestmark = pytest.mark.gpu

THRESHOLD = 1 << 16  # bytes


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30, offload_min_bytes=THRESHOLD)
    yield c
    c.destroy()


def cost(p):
    return p.n * (8 if p.kid == datagen.FMUL else 4)


def parts_around_threshold():
    sizes = {datagen.POLY: [0, 100, 16_383, 16_384, 100_003],
             datagen.FMUL: [7, 8_191, 8_192, 50_001],
             datagen.MC_PI: [3, 16_383, 16_384, 200_001]}
    parts, pid = [], 0
    for kid, ns in sizes.items():
        for n in ns:
            parts.append(datagen.make_part(kid, n, pid, with_data=kid != datagen.MC_PI))
            pid += 1
    return parts


def check_declined(g):
    assert g.status == sc.EDECLINED
    assert g.sum == 0.0 and g.max == -np.inf and g.count == 0 and g.n == 0


@pytest.mark.parametrize("mode", [sc.PER_LAUNCH, sc.BATCHED])
def test_reduce_declines_small_tasks(ctx, mode):
    parts = parts_around_threshold()
    d = DevParts(parts)
    per, tot = ctx.reduce(d.tasks, mode)
    kept = []
    for p, g in zip(parts, per):
        if cost(p) < THRESHOLD:
            check_declined(g)
        else:
            check_result(g, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
            kept.append(oracle_result(p))
    o = oracle.rdd_total(kept, datagen.SUM | datagen.MAX | datagen.COUNT)
    assert tot.n == o.n and tot.count == o.count and np.float32(tot.max) == np.float32(o.max)
    assert abs(tot.sum - o.sum) <= 1e-6 * abs(o.sum)


@pytest.mark.parametrize("mode", [sc.PER_LAUNCH, sc.BATCHED])
def test_map_partition_declines_small_tasks(ctx, mode):
    parts = [datagen.make_part(datagen.MC_PI, n, p, with_data=False)
             for p, n in enumerate([10, 16_383, 16_384, 300_001])]
    d = DevParts(parts)
    res = ctx.map_partition(d.tasks, mode)
    for p, g in zip(parts, res):
        if cost(p) < THRESHOLD:
            check_declined(g)
        else:
            check_result(g, oracle_result(p), p.kid, p.ops, f"n={p.n}")


def test_map_is_never_declined(ctx):
    p = datagen.make_part(datagen.FMUL, 100, 1)
    x, y = torch.from_numpy(p.x).cuda(), torch.from_numpy(p.y).cuda()
    out = torch.full((100,), float("nan"), device="cuda")
    ctx.map([sc.task(datagen.FMUL, 100, x, y, out, c=p.c)])
    torch.cuda.synchronize()
    want = oracle.fmul_map(p.x, p.y)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32))


def test_submit_declines_small_tasks(ctx):
    small = datagen.make_part(datagen.POLY, 1000, 0)
    big = datagen.make_part(datagen.POLY, 1 << 16, 1)
    d = DevParts([small, big])
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(d.tasks[0])
    assert e.value.code == sc.EDECLINED
    t = ctx.submit(d.tasks[1])
    deadline = time.time() + 10
    r = None
    while r is None and time.time() < deadline:
        r = ctx.poll(t)
    assert r is not None
    check_result(r, oracle_result(big), big.kid, big.ops, "served")
    ctx.serve_drain()


def test_offload_breakeven(ctx):
    slow = ctx.offload_breakeven(1e9)       # a 1 GB/s host path
    fast = ctx.offload_breakeven(2e9)
    assert 0 < slow < fast < (1 << 40)
    # break-even grows with the host rate and is unbounded once the host
    # streams as fast as HBM
    assert ctx.offload_breakeven(1e15) == 2 ** 64 - 1
    with pytest.raises(sc.SparkclError) as e:
        ctx.offload_breakeven(0.0)
    assert e.value.code == sc.EINVAL
    assert sc.strerror(sc.EDECLINED) == "declined by selective execution"
