"""GPU serving: continuous batching through sparkcl_submit / sparkcl_poll.

Each task's result must match the oracle, and must be bit-identical whether it
ran alone or in a mix with other tasks sharing the GPU.  Admission against a
small budget, oversize and invalid requests, executor relaunch after an idle
exit, the per-task-launch baseline mode, and the watchdog are covered too.
The watchdog case ends a long task from the host (stop word); every kernel
still exits normally.
"""
import ctypes
import math
import os
import threading
import time

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc
from gpu_helpers import DevParts, check_result, oracle_result

pytestmark = pytest.mark.gpu


def mixed_parts(count, seed, median=16384, lo=1024, hi=262144):
    sizes = datagen.lognormal_sizes(count, seed, 6, median, math.log(4.0), lo, hi)
    kids = datagen.uniform_kernel_ids(count, seed, 7)
    return [datagen.make_part(int(k), int(n), i, seed=0)
            for i, (n, k) in enumerate(zip(sizes, kids))]


# sparkcl_loadgen_run(ctx, tasks, sched_ns, count, lead_ns, stall_ms, &t0, done_ns,
# status, results)
LOADGEN_ARGS = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                ctypes.c_int64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64),
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]


def loadgen():
    lg = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(sc.__file__)),
                                  "libsparkcl_loadgen.so"))
    run = lg.sparkcl_loadgen_run
    run.restype = ctypes.c_int
    run.argtypes = LOADGEN_ARGS
    return run


def wait_all(ctx, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    pending = list(tickets)
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


def test_serve_matches_oracle(ctx):
    parts = mixed_parts(200, 11)
    d = DevParts(parts)
    tickets = [ctx.submit(t) for t in d.tasks]
    res = wait_all(ctx, tickets)
    for p, r in zip(parts, res):
        check_result(r, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
        assert r.t_arrive_ns <= r.t_admit_ns <= r.t_done_ns
    st = ctx.serve_stats()
    assert st["completed"] >= 200 and st["in_flight"] == 0 and st["pending"] == 0


def test_serve_alone_vs_mix_bit_identical(ctx):
    parts = mixed_parts(64, 12, median=65536, hi=1 << 20)
    d = DevParts(parts)
    alone = []
    for t in d.tasks[:16]:
        alone.append(wait_all(ctx, [ctx.submit(t)])[0])
    mix = wait_all(ctx, [ctx.submit(t) for t in d.tasks])
    for a, m in zip(alone, mix[:16]):
        assert key(a) == key(m)
    for p, m in zip(parts, mix):
        check_result(m, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")


def test_serve_concurrent_submitters(ctx):
    parts = mixed_parts(120, 13)
    d = DevParts(parts)
    results = [None] * len(parts)

    def worker(idx):
        tk = [(i, ctx.submit(d.tasks[i])) for i in idx]
        for (i, t), r in zip(tk, wait_all(ctx, [t for _, t in tk])):
            results[i] = r

    ths = [threading.Thread(target=worker, args=(list(range(k, len(parts), 4)),))
           for k in range(4)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    for p, r in zip(parts, results):
        check_result(r, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")


def test_serve_small_budget_waits():
    # a 6 MiB budget with ~1 MiB tasks: admission must queue and still finish
    c = sc.Context(device=0, arena_bytes=256 << 20, budget_bytes=6 << 20)
    try:
        parts = [datagen.make_part(datagen.FMUL, 131072 + i, i) for i in range(40)]
        d = DevParts(parts)
        res = wait_all(c, [c.submit(t) for t in d.tasks])
        for p, r in zip(parts, res):
            check_result(r, oracle_result(p), p.kid, p.ops, f"n={p.n}")
        st = c.serve_stats()
        assert st["budget_peak"] <= 6 << 20
        assert st["admission_waits"] > 0
        with pytest.raises(sc.SparkclError) as e:
            big = datagen.make_part(datagen.FMUL, 1 << 20, 99, with_data=False)
            x = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")
            c.submit(sc.task(sc.FMUL, 1 << 20, x, x))
        assert e.value.code == sc.ETOOBIG
        del big
    finally:
        c.destroy()


def test_serve_rejects_invalid(ctx):
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(7, 64, x))
    assert e.value.code == sc.ENOKERNEL
    with pytest.raises(sc.SparkclError) as e:
        ctx.submit(sc.task(sc.MC_PI, 64, ops=sc.SUM))
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.poll(1 << 60)
    assert e.value.code == sc.ENOTFOUND


def test_serve_per_task_launch_matches_resident(ctx):
    parts = mixed_parts(48, 14)
    d = DevParts(parts)
    resident = wait_all(ctx, [ctx.submit(t) for t in d.tasks])
    c = sc.Context(device=0, arena_bytes=256 << 20, flags=sc.FLAG_SERVE_PER_TASK)
    try:
        launched = wait_all(c, [c.submit(t) for t in d.tasks])
        assert c.serve_stats()["executor_launches"] >= len(parts)
    finally:
        c.destroy()
    for a, b in zip(resident, launched):
        assert key(a) == key(b)


def test_serve_relaunch_after_idle_exit():
    c = sc.Context(device=0, arena_bytes=256 << 20, idle_exit_ms=20)
    try:
        parts = mixed_parts(10, 15)
        d = DevParts(parts)
        first = wait_all(c, [c.submit(t) for t in d.tasks[:5]])
        time.sleep(0.3)  # the resident executor idles out
        second = wait_all(c, [c.submit(t) for t in d.tasks[5:]])
        assert c.serve_stats()["executor_launches"] >= 2
        for p, r in zip(parts, first + second):
            check_result(r, oracle_result(p), p.kid, p.ops, f"n={p.n}")
    finally:
        c.destroy()


def test_serve_watchdog_fails_long_task_then_recovers():
    # a 2^34-sample Monte-Carlo task (2^20 tiles) cannot finish within a 5 ms
    # watchdog; the host stops the executor (workers exit after their current
    # tile), fails the task with ETIMEDOUT, resets the device state and keeps
    # serving
    c = sc.Context(device=0, arena_bytes=256 << 20, watchdog_ms=5)
    try:
        t = c.submit(sc.task(sc.MC_PI, 1 << 34, pid=1))
        r = wait_all(c, [t], timeout=30)[0]
        assert r.status == sc.ETIMEDOUT
        parts = mixed_parts(8, 16, hi=65536)
        d = DevParts(parts)
        res = wait_all(c, [c.submit(x) for x in d.tasks])
        for p, q in zip(parts, res):
            check_result(q, oracle_result(p), p.kid, p.ops, f"n={p.n}")
    finally:
        c.destroy()


def test_native_load_generator_replays_a_trace(ctx):
    """The serving benchmark's load generator (libsparkcl_loadgen.so, over the
    public C ABI): a short trace is submitted at its scheduled times, every
    task completes with status OK after its scheduled arrival, and the results
    it collects match the oracle."""
    parts = mixed_parts(64, 5)
    d = DevParts(parts)
    count = 2000
    tasks = (sc.Task * count)(*[d.tasks[i % len(parts)] for i in range(count)])
    sched = (np.arange(count, dtype=np.int64) * 50_000)  # 20K tasks/s
    done = np.zeros(count, np.int64)
    status = np.full(count, -99, np.int32)
    run = loadgen()
    t0 = ctypes.c_int64()
    results = (sc.Result * count)()
    rc = run(ctx._h, ctypes.addressof(tasks), sched.ctypes.data, count, 5_000_000, 10_000,
             ctypes.byref(t0), done.ctypes.data, status.ctypes.data, ctypes.addressof(results))
    assert rc == 0
    assert np.all(status == 0)
    assert np.all(done >= t0.value + sched)
    want = [oracle_result(p) for p in parts]
    for i in range(count):
        p = parts[i % len(parts)]
        check_result(results[i], want[i % len(parts)], p.kid, p.ops, f"task {i} kid={p.kid} n={p.n}")
    # unsorted arrival times are refused
    bad = sched[::-1].copy()
    assert run(ctx._h, ctypes.addressof(tasks), bad.ctypes.data, count, 0, 1000,
               ctypes.byref(t0), done.ctypes.data, status.ctypes.data, None) == sc.EINVAL


@pytest.mark.parametrize("per_task,host", [(False, False), (True, False), (False, True)],
                         ids=["resident", "per_task_launch", "host_inputs"])
def test_serving_trace_at_full_rate_matches_oracle(per_task, host):
    """The serving workload as the benchmark runs it: Poisson arrivals at
    20K tasks/s (0.5 s, 10000 tasks), log-normal sizes of 1K to 4M elements
    (median 64K), uniform kernel ids, inputs at drawn offsets of a resident
    pool, a 64 GiB admission budget, replayed open-loop by the native load
    generator; every task completes with status OK and its element count, and
    a sample of 300 tasks plus the 20 largest match the oracle one by one.
    Both serving forms (the resident executor and one launch per task), and
    the resident executor with the pool in pinned host memory (each task's
    inputs staged over PCIe)."""
    import bench

    pool = 1 << 24
    x = datagen.x_for(datagen.FMUL, pool, 0, 0)   # N(0,1)
    y = datagen.y_for(datagen.FMUL, pool, 0, 0)   # U[0,2)
    if host:
        dx = torch.from_numpy(x).pin_memory()
        dy = torch.from_numpy(y).pin_memory()
    else:
        dx = torch.from_numpy(x).cuda()
        dy = torch.from_numpy(y).cuda()
    count = 10_000
    tr = datagen.serving_trace(count, rate=20000.0, pool=pool)
    tasks = bench.trace_tasks(sc, tr, dx.data_ptr(), dy.data_ptr(), host=host)
    sched = np.ascontiguousarray((tr.t_arrive * 1e9).astype(np.int64))
    done = np.zeros(count, np.int64)
    status = np.full(count, -99, np.int32)
    results = (sc.Result * count)()
    c = sc.Context(device=0, arena_bytes=(4 << 30) if host else (1 << 30),
                   budget_bytes=64 << 30, flags=sc.FLAG_SERVE_PER_TASK if per_task else 0)
    try:
        t0 = ctypes.c_int64()
        rc = loadgen()(c._h, tasks.ctypes.data, sched.ctypes.data, count, 20_000_000, 10_000,
                       ctypes.byref(t0), done.ctypes.data, status.ctypes.data,
                       ctypes.addressof(results))
    finally:
        c.destroy()
    assert rc == 0
    assert np.all(status == 0)
    assert [results[i].n for i in range(count)] == [int(v) for v in tr.sizes]
    rng = np.random.default_rng(5)
    pick = set(rng.choice(count, 300, replace=False).tolist())
    pick |= set(np.argsort(tr.sizes)[-20:].tolist())
    for i in sorted(pick):
        kid, n, off = int(tr.kids[i]), int(tr.sizes[i]), int(tr.offsets[i])
        if kid == datagen.MC_PI:
            o = oracle.run_task(kid, sc.COUNT, n, None, None, seed=0, pid=i)
            ops = sc.COUNT
        else:
            ops = sc.SUM | sc.MAX
            o = oracle.run_task(kid, ops, n, x[off:off + n],
                                y[off:off + n] if kid == datagen.FMUL else None,
                                coef=datagen.POLY_COEF if kid == datagen.POLY else (),
                                c=datagen.FMUL_C)
        check_result(results[i], o, kid, ops, f"task {i} kid={kid} n={n} off={off}")


def test_serve_light_load_keeps_claimed_tickets():
    # Regression: one single-tile task every ~5 ms for ~0.5 s with a 20 ms
    # idle period.  The dispatcher stays alive (arrivals come faster than its
    # idle exit), while the workers holding the highest tickets wait for
    # ~100 tasks, far past any multiple of the idle period.  A worker that
    # gave up its claimed ticket would strand that tile: its task would never
    # complete and the 2 s watchdog would fail it with ETIMEDOUT.
    c = sc.Context(device=0, arena_bytes=256 << 20, idle_exit_ms=20, watchdog_ms=2000)
    try:
        parts = [datagen.make_part(datagen.POLY if i % 2 else datagen.FMUL, 1000 + i, i)
                 for i in range(100)]
        d = DevParts(parts)
        tickets = []
        for t in d.tasks:
            tickets.append(c.submit(t))
            time.sleep(0.005)
        res = wait_all(c, tickets, timeout=30)
        for p, r in zip(parts, res):
            check_result(r, oracle_result(p), p.kid, p.ops, f"kid={p.kid} n={p.n}")
        assert c.serve_stats()["failed"] == 0
    finally:
        c.destroy()


def test_serve_tuning_change_while_tasks_wait():
    # A task keeps the tile size chosen when it was submitted: tasks still
    # waiting for a ring slot when the serving tile table changes must cover
    # exactly their n elements (samples) and match the oracle; tasks submitted
    # after the change use the new table and match the oracle too.  Per-task
    # launches over a two-slot ring keep most of the tasks waiting.
    c = sc.Context(device=0, arena_bytes=256 << 20, ring_capacity=2,
                   flags=sc.FLAG_SERVE_PER_TASK)
    try:
        parts = [datagen.make_part(datagen.MC_PI, (1 << 26) + 3 * i, i, with_data=False)
                 for i in range(24)]
        parts += [datagen.make_part(datagen.FMUL, (1 << 20) + 5 * i, 100 + i)
                  for i in range(8)]
        d = DevParts(parts)
        first = [c.submit(t) for t in d.tasks]
        before = c.serve_stats()
        t = c.get_tuning()
        for k in range(3):
            for b in range(len(t.tile[2][k])):
                t.tile[2][k][b] = 1 << 12
        c.set_tuning(t)
        later = [c.submit(t) for t in d.tasks]
        res = wait_all(c, first + later, timeout=60)
        # the oracle once per partition, partitions side by side (the C
        # oracle releases the GIL)
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(16) as ex:
            want = list(ex.map(oracle_result, parts))
        for i, r in enumerate(res):
            p = parts[i % len(parts)]
            check_result(r, want[i % len(parts)], p.kid, p.ops, f"#{i} kid={p.kid} n={p.n}")
        assert before["pending"] + before["in_flight"] > 0
    finally:
        c.destroy()
