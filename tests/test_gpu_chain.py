"""Fused map chains (map -> map -> ... -> reduce in one pass, sec. 3.1.3):
sparkcl_reduce_chain against the oracle's maps composed stage by stage --
bit-exact materialised outputs, sums within the FP64 bar, exact max."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, check_total

pytestmark = pytest.mark.gpu

STAGES = [(0.5, -0.25, 0.125), (1.0, 2.0), (0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0 / 64)]


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.destroy()


def want(p, stages):
    v = oracle.chain_map(p.x, p.y, p.kid, p.coef, np.float32(p.c), stages)
    return v, oracle.Result(sum=oracle.fsum(v) if p.ops & datagen.SUM else 0.0,
                            max=oracle.fmax(v) if p.ops & datagen.MAX else -np.inf,
                            count=0, n=p.n)


@pytest.mark.parametrize("nst", [0, 1, 2, 3])
@pytest.mark.parametrize("off", [0, 1])
def test_chain_matches_composed_oracle(ctx, nst, off):
    stages = STAGES[:nst]
    parts = [datagen.make_part(k, n, i) for i, (k, n) in
             enumerate([(datagen.FMUL, 1), (datagen.POLY, 4097), (datagen.FMUL, 100_003),
                        (datagen.POLY, 262_147), (datagen.FMUL, 1 << 20)])]
    d = DevParts(parts, off, off, out=True)
    per, tot = ctx.reduce_chain(d.tasks, [sc.stage(s) for s in stages])
    torch.cuda.synchronize()
    for p, g, o in zip(parts, per, d.outs):
        v, r = want(p, stages)
        check_result(g, r, p.kid, p.ops, f"kid={p.kid} n={p.n} stages={nst}")
        assert np.array_equal(o.cpu().numpy().view(np.uint32), v.view(np.uint32))


def test_empty_chain_equals_plain_reduce(ctx):
    parts = [datagen.make_part(datagen.FMUL, 300_001, 3), datagen.make_part(datagen.POLY, 77_777, 4)]
    d = DevParts(parts)
    a, ta = ctx.reduce_chain(d.tasks, [])
    b, tb = ctx.reduce(d.tasks, sc.BATCHED)
    for x, y in zip(a, b):
        assert (x.sum, x.max, x.n) == (y.sum, y.max, y.n)


def test_chain_is_part_of_the_plan_key(ctx):
    p = datagen.make_part(datagen.POLY, 50_000, 7)
    d = DevParts([p])
    r1, _ = ctx.reduce_chain(d.tasks, [sc.stage((1.0, 2.0))])
    r2, _ = ctx.reduce_chain(d.tasks, [sc.stage((0.0, 3.0))])
    _, w1 = want(p, [(1.0, 2.0)])
    _, w2 = want(p, [(0.0, 3.0)])
    check_result(r1[0], w1, p.kid, p.ops, "first chain")
    check_result(r2[0], w2, p.kid, p.ops, "second chain")


def test_chain_errors(ctx):
    p = datagen.make_part(datagen.POLY, 1000, 0)
    d = DevParts([p])
    bad = sc.stage((1.0, 2.0))
    bad.kernel_id = sc.FMUL
    deg = sc.stage((1.0,) * 8)
    deg.degree = 8
    for stages in ([sc.stage((1.0,))] * 5, [bad], [deg]):
        with pytest.raises(sc.SparkclError) as e:
            ctx.reduce_chain(d.tasks, stages)
        assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_chain([sc.task(sc.MC_PI, 100)], [])
    assert e.value.code == sc.EINVAL


def test_chain_full_size(ctx):
    # The 64 x 2^22 FMUL RDD (x~N(0,1), y~U[0,2)) through FMUL -> POLY2 ->
    # POLY1, reduced without materialising anything: the fused chain at full
    # size in the launch configuration the benchmark times (the chain rule's
    # occupancy, the per-launch tiles that follow from it).  Every partition's
    # SUM and MAX against the oracle's composed maps, and the RDD total.
    parts = datagen.fmul_rdd()
    d = DevParts(parts)
    stages = STAGES[:2]
    per, tot = ctx.reduce_chain(d.tasks, [sc.stage(s) for s in stages])
    torch.cuda.synchronize()
    results = [want(p, stages)[1] for p in parts]
    for p, g, o in zip(parts, per, results):
        check_result(g, o, p.kid, p.ops, f"pid={p.pid}")
    check_total(tot, results, datagen.SUM | datagen.MAX)
