"""GPU serving of host-resident partitions (SPARKCL_TASK_HOST_INPUT through
sparkcl_submit): the server stages each task's inputs into the arena over PCIe
while other tasks run, and the task takes a ring slot once its copy is done.

A served host-input task must give bit-identically the result of the same data
served from device memory at the same 16-byte alignment (same tiles, same
summation order), within the oracle's tolerance, alone and in a mix with
device tasks; admission must charge the staging bytes against the budget; and
pageable memory, Monte-Carlo tasks and map outputs are refused.
"""
import math
import time

import numpy as np
import pytest
import torch

import datagen
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, oracle_result

pytestmark = pytest.mark.gpu


def pinned(a: np.ndarray, offset: int) -> torch.Tensor:
    """Pinned host copy of a float32 array, `offset` floats into its allocation."""
    buf = torch.empty(a.size + offset + 4, dtype=torch.float32).pin_memory()
    view = buf[offset:offset + a.size]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return view


class HostParts:
    """Pinned host copies of streaming partitions and their host-input tasks."""

    def __init__(self, parts, offsets):
        self.keep, self.tasks = [], []
        for p, off in zip(parts, offsets):
            x = pinned(p.x, off)
            y = pinned(p.y, (off + 1) % 4) if p.y is not None else None
            self.keep += [x, y]
            self.tasks.append(sc.task(p.kid, p.n, x, y, ops=p.ops, coef=p.coef, c=p.c,
                                      host=True))


def device_twins(parts, offsets):
    """Device copies at the same float offsets (so the same 16-byte alignment)."""
    out = []
    for p, off in zip(parts, offsets):
        d = DevParts([p], xoff=off, yoff=(off + 1) % 4)
        out.append(d)
    return out


def stream_parts(count, seed, median=65536, lo=1, hi=1 << 20):
    sizes = datagen.lognormal_sizes(count, seed, 6, median, math.log(4.0), lo, hi)
    kids = [datagen.POLY if i % 2 else datagen.FMUL for i in range(count)]
    return [datagen.make_part(k, int(n), i, seed=0) for i, (n, k) in enumerate(zip(sizes, kids))]


def wait_all(ctx, tickets, timeout=60.0):
    out, pending, t0 = {}, list(tickets), time.time()
    while pending:
        rest = []
        for t in pending:
            r = ctx.poll(t)
            if r is None:
                rest.append(t)
            else:
                out[t] = r
        pending = rest
        if pending:
            assert time.time() - t0 < timeout, f"{len(pending)} tasks not done"
            time.sleep(0.0002)
    return [out[t] for t in tickets]


def key(r):
    return (r.sum, float(r.max), r.count, r.n, r.status)


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.destroy()


def test_host_input_matches_device_and_oracle(ctx):
    parts = stream_parts(40, 21) + [datagen.make_part(datagen.FMUL, 3, 90),
                                    datagen.make_part(datagen.POLY, 4097, 91)]
    offs = [i % 4 for i in range(len(parts))]
    h = HostParts(parts, offs)
    twins = device_twins(parts, offs)
    host_res = wait_all(ctx, [ctx.submit(t) for t in h.tasks])
    dev_res = wait_all(ctx, [ctx.submit(d.tasks[0]) for d in twins])
    for p, a, b in zip(parts, host_res, dev_res):
        assert key(a) == key(b), f"kid={p.kid} n={p.n}"
        check_result(a, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
        assert a.t_arrive_ns <= a.t_admit_ns <= a.t_done_ns


def test_host_input_alone_vs_mix(ctx):
    hparts = stream_parts(24, 22, median=262144, hi=1 << 21)
    offs = [(3 * i) % 4 for i in range(len(hparts))]
    h = HostParts(hparts, offs)
    alone = [wait_all(ctx, [ctx.submit(t)])[0] for t in h.tasks[:8]]
    # the mix: host-input tasks interleaved with device and Monte-Carlo tasks
    dparts = [datagen.make_part(k, 50_000 + 977 * i, 100 + i)
              for i, k in enumerate([datagen.POLY, datagen.FMUL, datagen.MC_PI] * 8)]
    d = DevParts(dparts)
    order = []
    for i in range(max(len(h.tasks), len(d.tasks))):
        if i < len(h.tasks):
            order.append(("h", i))
        if i < len(d.tasks):
            order.append(("d", i))
    tickets = [ctx.submit(h.tasks[i] if s == "h" else d.tasks[i]) for s, i in order]
    res = dict(zip(order, wait_all(ctx, tickets)))
    for i, a in enumerate(alone):
        assert key(a) == key(res[("h", i)])
    for i, p in enumerate(hparts):
        check_result(res[("h", i)], oracle_result(p), p.kid, p.ops, f"host kid={p.kid} n={p.n}")
    for i, p in enumerate(dparts):
        check_result(res[("d", i)], oracle_result(p), p.kid, p.ops, f"dev kid={p.kid} n={p.n}")


def test_host_input_small_budget_waits():
    # 8 MiB budget, FMUL tasks of ~2 MiB staging each: admission queues on the
    # staging bytes and still finishes every task
    c = sc.Context(device=0, arena_bytes=256 << 20, budget_bytes=8 << 20)
    try:
        parts = [datagen.make_part(datagen.FMUL, 250_000 + 13 * i, i) for i in range(24)]
        h = HostParts(parts, [i % 4 for i in range(len(parts))])
        res = wait_all(c, [c.submit(t) for t in h.tasks])
        for p, r in zip(parts, res):
            check_result(r, oracle_result(p), p.kid, p.ops, f"n={p.n}")
        st = c.serve_stats()
        assert st["budget_peak"] <= 8 << 20
        assert st["admission_waits"] > 0
        assert st["in_flight"] == 0 and st["budget_in_use"] == 0
    finally:
        c.destroy()


def test_host_input_per_task_launch_matches_resident(ctx):
    parts = stream_parts(16, 23)
    h = HostParts(parts, [1] * len(parts))
    resident = wait_all(ctx, [ctx.submit(t) for t in h.tasks])
    c = sc.Context(device=0, arena_bytes=256 << 20, flags=sc.FLAG_SERVE_PER_TASK)
    try:
        launched = wait_all(c, [c.submit(t) for t in h.tasks])
    finally:
        c.destroy()
    for a, b in zip(resident, launched):
        assert key(a) == key(b)


def test_host_input_empty_and_refused(ctx):
    x = torch.zeros(64, dtype=torch.float32).pin_memory()
    r = wait_all(ctx, [ctx.submit(sc.task(sc.POLY, 0, x, coef=(1.0,), host=True))])[0]
    assert r.status == 0 and r.n == 0 and r.sum == 0.0 and r.max == -np.inf
    pageable = np.zeros(64, dtype=np.float32)
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(sc.POLY, 64, pageable, coef=(1.0,), host=True))
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(sc.FMUL, 64, x, pageable, host=True))
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(sc.MC_PI, 64, host=True))
    assert e.value.code == sc.EINVAL
    out = torch.empty(64, dtype=torch.float32, device="cuda")
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(sc.POLY, 64, x, out=out, coef=(1.0,), host=True))
    assert e.value.code == sc.EINVAL
    # serving still works after the refusals
    r = wait_all(ctx, [ctx.submit(sc.task(sc.POLY, 64, x, coef=(2.0,), host=True))])[0]
    assert r.status == 0 and r.n == 64 and r.sum == 128.0
