"""Graph replay of the batched path: SPARKCL_GRAPH (the persistent executor
captured once into a hipGraph kept with the cached plan, replayed per call)
and capture of the asynchronous call into a caller's own graph.

Each replay must recompute from the inputs as they are at replay time: the
inputs are changed by eager work between replays, and every replay is
compared with an eager BATCHED call on the same inputs (the same tile
decomposition, so bit-identical) and, once, with the oracle.  No memset is
recorded in any graph; the executor leaves its own counters at zero.
"""
import math

import numpy as np
import pytest
import torch

import datagen
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, oracle_result

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.destroy()


def mixed_parts(count, seed):
    sizes = datagen.lognormal_sizes(count, seed, seed + 1, 8192, math.log(4.0), 16, 300_000)
    kids = datagen.uniform_kernel_ids(count, seed, seed + 2)
    return [datagen.make_part(int(k), int(n), 1000 * seed + i)
            for i, (n, k) in enumerate(zip(sizes, kids))]


def key(r):
    return (r.sum, float(np.float32(r.max)), r.count, r.n, r.status)


def decode(buf, count):
    raw = buf.cpu().numpy()
    return [sc.Result.from_buffer_copy(raw[64 * i:64 * (i + 1)].tobytes()) for i in range(count)]


def scale_inputs(d, f):
    for t in d.keep:
        if t is not None:
            t.mul_(f)


def test_graph_mode_replays_track_inputs(ctx):
    parts = mixed_parts(200, 3)
    d = DevParts(parts)
    for rep in range(4):
        g, gt = ctx.reduce(d.tasks, sc.GRAPH)
        b, bt = ctx.reduce(d.tasks, sc.BATCHED)
        assert [key(r) for r in g] == [key(r) for r in b], f"replay {rep}"
        assert key(gt) == key(bt), f"replay {rep}"
        if rep == 0:
            for p, r in zip(parts, g):
                check_result(r, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
        scale_inputs(d, 0.5)  # eager work between replays
        torch.cuda.synchronize()


def test_graph_mode_async_back_to_back(ctx):
    parts = mixed_parts(64, 5)
    d = DevParts(parts)
    want, wt = ctx.reduce(d.tasks, sc.BATCHED)
    dres = torch.zeros(64 * len(parts), dtype=torch.uint8, device="cuda")
    dtot = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for _ in range(5):
        ctx.reduce_async(d.tasks, sc.GRAPH, dres, dtot)
    torch.cuda.synchronize()
    assert [key(r) for r in decode(dres, len(parts))] == [key(r) for r in want]
    assert key(decode(dtot, 1)[0]) == key(wt)


@pytest.mark.parametrize("mode", [sc.PER_LAUNCH, sc.BATCHED, sc.GRAPH])
def test_caller_capture_replays(ctx, mode):
    parts = mixed_parts(48, 7 + mode)
    d = DevParts(parts)
    n = len(parts)
    dres = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
    dtot = torch.zeros(64, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ctx.reduce_async(d.tasks, mode, dres, dtot, stream=s)  # caches the plan
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        ctx.reduce_async(d.tasks, mode, dres, dtot, stream=torch.cuda.current_stream())
    for rep in range(4):
        dres.fill_(0xAB)  # eager work between replays; stale results must not survive
        dtot.fill_(0xAB)
        graph.replay()
        torch.cuda.synchronize()
        want, wt = ctx.reduce(d.tasks, sc.BATCHED)
        got = decode(dres, n)
        assert [key(r) for r in got] == [key(r) for r in want], f"mode {mode} replay {rep}"
        assert key(decode(dtot, 1)[0]) == key(wt), f"mode {mode} replay {rep}"
        if rep == 0:
            for p, r in zip(parts, got):
                check_result(r, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
        scale_inputs(d, 2.0)
        torch.cuda.synchronize()
    del graph


def test_capture_needs_a_cached_plan(ctx):
    cached = DevParts(mixed_parts(8, 11))
    fresh = DevParts(mixed_parts(9, 13))
    dres = torch.zeros(64 * 8, dtype=torch.uint8, device="cuda")
    other = torch.zeros(64 * 9, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ctx.reduce_async(cached.tasks, sc.BATCHED, dres, None, stream=s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        cs = torch.cuda.current_stream()
        with pytest.raises(sc.SparkclError) as e1:
            ctx.reduce_async(fresh.tasks, sc.BATCHED, other, None, stream=cs)
        with pytest.raises(sc.SparkclError) as e2:
            ctx.reduce(cached.tasks, sc.BATCHED, stream=cs)
        ctx.reduce_async(cached.tasks, sc.BATCHED, dres, None, stream=cs)
    assert e1.value.code == sc.EINVAL and e2.value.code == sc.EINVAL
    dres.zero_()
    graph.replay()
    torch.cuda.synchronize()
    want, _ = ctx.reduce(cached.tasks, sc.BATCHED)
    assert [key(r) for r in decode(dres, 8)] == [key(r) for r in want]
    del graph


def test_graph_mode_rejects_host_input(ctx):
    x = np.ones(1000, dtype=np.float32)
    t = sc.task(sc.POLY, 1000, x, coef=(0.0, 1.0), host=True)
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce([t], sc.GRAPH)
    assert e.value.code == sc.EINVAL
    r, _ = ctx.reduce([t], sc.BATCHED)
    assert r[0].sum == 1000.0
