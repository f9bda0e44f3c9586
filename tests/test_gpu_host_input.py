"""Host-resident partitions: inputs in host memory streamed through the
library's staging ring (host-to-device copies overlapped with the kernels),
against the same data reduced from device memory (bit-identical, same tiles)
and against the oracle."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc
from gpu_helpers import check_result, oracle_result

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.destroy()


def pinned_copy(a: np.ndarray, off: int = 0) -> torch.Tensor:
    """A pinned host tensor holding `a` starting `off` elements in."""
    buf = torch.empty(a.size + off + 4, dtype=torch.float32).pin_memory()
    buf[off:off + a.size].copy_(torch.from_numpy(a))
    return buf[off:off + a.size]


def same(a, b):
    return (a.sum, a.max, a.count, a.n, a.status) == (b.sum, b.max, b.count, b.n, b.status)


SIZES = [(datagen.POLY, 0), (datagen.FMUL, 1), (datagen.POLY, 3), (datagen.FMUL, 4097),
         (datagen.POLY, 100_003), (datagen.FMUL, 1 << 20), (datagen.POLY, 262_147),
         (datagen.FMUL, 777_777)]


@pytest.mark.parametrize("xoff,yoff", [(0, 0), (1, 1), (2, 3)])
def test_host_input_matches_device_input_and_oracle(ctx, xoff, yoff):
    parts = [datagen.make_part(k, n, i) for i, (k, n) in enumerate(SIZES)]
    keep, htasks, dtasks = [], [], []
    for p in parts:
        hx = pinned_copy(p.x, xoff)
        hy = pinned_copy(p.y, yoff) if p.y is not None else None
        dx, dy = hx.cuda(), (hy.cuda() if hy is not None else None)
        keep += [hx, hy, dx, dy]
        kw = dict(ops=p.ops, coef=p.coef, c=p.c)
        htasks.append(sc.task(p.kid, p.n, hx, hy, host=True, **kw))
        # the device copy keeps the host offsets' 16-byte alignment
        dbuf_x = torch.empty(p.n + xoff + 4, device="cuda")[xoff:xoff + p.n]
        dbuf_x.copy_(dx)
        dbuf_y = None
        if dy is not None:
            dbuf_y = torch.empty(p.n + yoff + 4, device="cuda")[yoff:yoff + p.n]
            dbuf_y.copy_(dy)
        keep += [dbuf_x, dbuf_y]
        dtasks.append(sc.task(p.kid, p.n, dbuf_x, dbuf_y, **kw))
    hper, htot = ctx.reduce(htasks, sc.BATCHED)      # mode is ignored for host inputs
    dper, dtot = ctx.reduce(dtasks, sc.PER_LAUNCH)
    for p, h, d in zip(parts, hper, dper):
        assert same(h, d), (p.kid, p.n)
        check_result(h, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
    assert same(htot, dtot)


def test_pageable_numpy_inputs_and_reuse(ctx):
    p = datagen.make_part(datagen.FMUL, 300_001, 3)
    x, y = p.x.copy(), p.y.copy()
    tasks = [sc.task(datagen.FMUL, p.n, x, y, ops=p.ops, c=p.c, host=True)]
    per, _ = ctx.reduce(tasks)
    check_result(per[0], oracle_result(p), p.kid, p.ops, "pageable")
    # same plan, new contents: the copies happen on every call
    x *= np.float32(2.0)
    per2, _ = ctx.reduce(tasks)
    q = datagen.Part(kid=p.kid, ops=p.ops, n=p.n, pid=p.pid, x=x, y=y, c=p.c)
    check_result(per2[0], oracle_result(q), p.kid, p.ops, "reused plan")


def test_async_host_input(ctx):
    parts = [datagen.make_part(datagen.POLY, 50_000 + i, i) for i in range(5)]
    hx = [pinned_copy(p.x) for p in parts]
    tasks = [sc.task(p.kid, p.n, h, ops=p.ops, coef=p.coef, host=True) for p, h in zip(parts, hx)]
    dres = torch.zeros(64 * len(parts), dtype=torch.uint8, device="cuda")
    ctx.reduce_async(tasks, sc.PER_LAUNCH, dres)
    torch.cuda.synchronize()
    raw = dres.cpu().numpy()
    for i, p in enumerate(parts):
        g = sc.Result.from_buffer_copy(raw[64 * i:64 * (i + 1)].tobytes())
        check_result(g, oracle_result(p), p.kid, p.ops, f"async {i}")


def test_host_input_errors(ctx):
    p = datagen.make_part(datagen.POLY, 1000, 0)
    hx = pinned_copy(p.x)
    dx = hx.cuda()
    h = sc.task(p.kid, p.n, hx, coef=p.coef, host=True)
    d = sc.task(p.kid, p.n, dx, coef=p.coef)
    for bad in ([h, d],                                                   # mixed
                [sc.task(sc.MC_PI, 100, host=True)],                      # nothing to stream
                [sc.task(p.kid, p.n, hx, out=dx, coef=p.coef, host=True)]):  # out set
        with pytest.raises(sc.SparkclError) as e:
            ctx.reduce(bad)
        assert e.value.code == sc.EINVAL
    # served host-input tasks must sit in pinned memory (the serving thread
    # copies them asynchronously); pageable memory is refused at submit
    pageable = torch.from_numpy(p.x.copy())
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(p.kid, p.n, pageable, coef=p.coef, host=True))
    assert e.value.code == sc.EINVAL
    t = sc.task(p.kid, p.n, hx, coef=p.coef, host=True)
    t.flags = 2
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce([t])
    assert e.value.code == sc.EINVAL
