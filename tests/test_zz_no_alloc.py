"""The allocation-free ReduceCL entry point (sparkcl_reduce_noalloc) against
the batched sparkcl_reduce_async it mirrors, through the C ABI: two calls in a
row, the second with a smaller input, each bit-identical to the existing
entry point on the same tasks and within the oracle's bar; then its limits."""
import math

import numpy as np
import pytest
import torch

import datagen
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, check_total, oracle_result

pytestmark = pytest.mark.gpu


def results(dres, dtot, n):
    torch.cuda.synchronize()
    raw = dres.cpu().numpy()
    per = [sc.Result.from_buffer_copy(raw[64 * i:64 * (i + 1)].tobytes()) for i in range(n)]
    tot = sc.Result.from_buffer_copy(dtot.cpu().numpy().tobytes())
    return per, tot


def key(r):
    return (r.sum, float(r.max), r.count, r.n, r.status)


def both(ctx, tasks):
    n = len(tasks)
    a_res = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
    a_tot = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b_res = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
    b_tot = torch.zeros(64, dtype=torch.uint8, device="cuda")
    ctx.reduce_noalloc(tasks, a_res, a_tot)
    ctx.reduce_async(tasks, sc.BATCHED, b_res, b_tot)
    return results(a_res, a_tot, n), results(b_res, b_tot, n)


def check_call(ctx, parts):
    d = DevParts(parts)
    (per, tot), (ref, rtot) = both(ctx, d.tasks)
    want = [oracle_result(p) for p in parts]
    for p, g, r, o in zip(parts, per, ref, want):
        where = f"kid={p.kid} n={p.n} pid={p.pid}"
        assert key(g) == key(r), where
        check_result(g, o, p.kid, p.ops, where)
    ops = 0
    for p in parts:
        ops |= p.ops
    assert (tot.sum, tot.max, tot.count, tot.n) == (rtot.sum, rtot.max, rtot.count, rtot.n)
    check_total(tot, want, ops)


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.destroy()


def test_two_calls_second_smaller(ctx):
    # 1: 700 mixed tasks spread over many sizes (the mixed-batch cut), with
    #    edge sizes; 2: a smaller call whose tasks and tiles sit inside the
    #    first call's regions of the array, so stale tickets, partials or
    #    results from call 1 would show
    sizes = datagen.lognormal_sizes(700, 21, 3, 16384, math.log(4.0), 1, 1 << 20)
    kids = datagen.uniform_kernel_ids(700, 21, 4)
    first = [datagen.make_part(int(k), int(n), i) for i, (n, k) in enumerate(zip(sizes, kids))]
    first += [datagen.make_part(k, n, 700 + i) for i, (k, n) in
              enumerate([(1, 0), (2, 1), (3, 1), (1, 4097), (2, 65537), (3, (1 << 20) + 1)])]
    check_call(ctx, first)
    second = [datagen.make_part(int(k), int(n) // 3 + 1, i)
              for i, (n, k) in enumerate(zip(sizes[:40], kids[:40]))]
    check_call(ctx, second)


@pytest.mark.parametrize("workload", ["rdd_64x2p22", "uneven_4096"])
def test_full_size_batches(ctx, workload):
    # the two batched workloads at their full sizes: the 64 x 2^22 FMUL RDD
    # (512 tiles) and the 4096-partition uneven batch of mixed kernels (the
    # mixed-batch cut, about 14000 tiles), each bit-identical to the batched
    # call and within the oracle's bar, with the RDD total
    parts = datagen.fmul_rdd() if workload == "rdd_64x2p22" else datagen.uneven_rdd()
    check_call(ctx, parts)


def test_repeated_calls_and_per_task_only(ctx):
    parts = [datagen.make_part(k, 200_000 + 7 * i, i) for i, k in enumerate([1, 2, 3] * 5)]
    d = DevParts(parts)
    n = len(parts)
    keys = []
    for _ in range(3):
        dres = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
        dtot = torch.zeros(64, dtype=torch.uint8, device="cuda")
        ctx.reduce_noalloc(d.tasks, dres, dtot)
        per, tot = results(dres, dtot, n)
        keys.append([key(r) for r in per] + [(tot.sum, tot.max, tot.count, tot.n)])
    assert keys[0] == keys[1] == keys[2]
    # per-task results only: the RDD total is not computed
    dres = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
    ctx.reduce_noalloc(d.tasks, dres, None)
    per, _ = results(dres, torch.zeros(64, dtype=torch.uint8, device="cuda"), n)
    assert [key(r) for r in per] == keys[0][:n]
    for p, g in zip(parts, per):
        check_result(g, oracle_result(p), p.kid, p.ops, f"kid={p.kid}")


def test_limits(ctx):
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    dres = torch.zeros(64 * 8193, dtype=torch.uint8, device="cuda")
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_noalloc([sc.task(sc.POLY, 16, x, coef=(1.0,))] * 8193, dres)
    assert e.value.code == sc.ETOOBIG
    # more tiles than the array holds: two 2^40-sample Monte-Carlo tasks are
    # at least 2^19 tiles under any tile size (at most 2^22)
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_noalloc([sc.task(sc.MC_PI, 1 << 40, pid=1)] * 2, dres)
    assert e.value.code == sc.ETOOBIG
    hx = torch.zeros(16, dtype=torch.float32).pin_memory()
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_noalloc([sc.task(sc.POLY, 16, hx, coef=(1.0,), host=True)], dres)
    assert e.value.code == sc.EINVAL
    # the entry point still works after its errors
    dres = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dtot = torch.zeros(64, dtype=torch.uint8, device="cuda")
    ctx.reduce_noalloc([sc.task(sc.POLY, 16, x, coef=(2.0,))], dres, dtot)
    per, tot = results(dres, dtot, 1)
    assert per[0].sum == 32.0 and tot.sum == 32.0 and per[0].status == 0
