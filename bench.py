"""Benchmark of the SparkCL map -> reduce hot path on one MI355X.

Step = one ReduceCL pass (paper sec. 3.1.3) over the 64-partition RDD: 64
partitions x 2^22 float32 pairs (x ~ N(0,1), y ~ U[0,2), seeded per
partition), FMUL map z = x*y + 0.1x fused with per-partition SUM and MAX and
the RDD-level combine, run as one persistent-executor launch over the device
tile queue of a cached plan, tile sizes from the tuning table.  Inputs are resident in HBM before timing starts.  The metric is
elements/s; the roofline object reports the executor kernel's algorithmic HBM
bandwidth (8 B per element) against the 8 TB/s peak.

Extras (same process, untimed relative to the step): the same RDD with one
launch per partition, the single 2^20 POLY partition, the 256 x 2^24 Monte-Carlo
partitions, the 4096-partition uneven batch (persistent vs per-partition),
the array-valued ReduceCL (vector add) over the resident x tensor, and the
Poisson serving stream (resident executor vs one launch per task).

Run: python bench.py [--steps K] [--warmup W] [--no-extras] [--serve-seconds S]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import statistics
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ = 256, 2.4
ALU_PEAK_TOPS = CUS * 64 * CLOCK_GHZ / 1e3  # 32-bit VALU lane-ops, T/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1505_01120_amd", "csrc", "kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_isa():
    """Resource figures of the library's compiled device code (written by the build
    next to the library), if they belong to the current kernel source."""
    p = os.path.join(ROOT, "paper_1505_01120_amd", "isa.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return d if d.get("kernels_sha256_16") == kernel_source_hash() else None


def load_traffic(kind: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(kind)
    if not e or e.get("kernel_source") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


class Resident:
    """The 64-partition RDD resident in HBM: one x and one y tensor, each
    partition a contiguous 16-byte-aligned slice."""

    def __init__(self, parts: int, n: int):
        import torch

        import datagen
        self.parts, self.n = parts, n
        self.x = torch.empty(parts * n, dtype=torch.float32, device="cuda")
        self.y = torch.empty(parts * n, dtype=torch.float32, device="cuda")
        hx = torch.empty(n, dtype=torch.float32).pin_memory()
        hy = torch.empty(n, dtype=torch.float32).pin_memory()
        for p in range(parts):
            datagen.fill(n, 0, p, 1, datagen.NORMAL, out=hx.numpy())
            datagen.fill(n, 0, p, 2, datagen.U_02, out=hy.numpy())
            self.x[p * n:(p + 1) * n].copy_(hx)
            self.y[p * n:(p + 1) * n].copy_(hy)
        torch.cuda.synchronize()

    def pinned(self):
        """Pinned host copies of x and y (made once): the host-resident form
        of the same RDD."""
        import torch
        if getattr(self, "hx", None) is None:
            self.hx = torch.empty(self.parts * self.n, dtype=torch.float32).pin_memory()
            self.hy = torch.empty(self.parts * self.n, dtype=torch.float32).pin_memory()
            self.hx.copy_(self.x)
            self.hy.copy_(self.y)
        return self.hx, self.hy

    def tasks(self, sc, kid=None):
        import datagen
        out = []
        for p in range(self.parts):
            xs = self.x[p * self.n:(p + 1) * self.n]
            ys = self.y[p * self.n:(p + 1) * self.n]
            out.append(sc.task(sc.FMUL, self.n, xs, ys, ops=sc.SUM | sc.MAX,
                               pid=p, c=datagen.FMUL_C))
        return out


def time_async(ctx, sc, tasks, mode, steps, warmup, dres, dtot):
    """(wall ms per step, event ms per step) of back-to-back async reduces.
    The batch is converted to a task array once, as a caller replaying it
    would keep it."""
    import torch
    if not isinstance(tasks, sc.TaskArray):
        tasks = sc.task_array(tasks)
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.reduce_async(tasks, mode, dres, dtot, stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        ctx.reduce_async(tasks, mode, dres, dtot, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, e0.elapsed_time(e1) / steps


def spot_check(ctx, sc, res: Resident, tasks, pids=(0, 33, 63)):
    """Untimed: blocking reduce against the oracle on a few partitions."""
    import numpy as np

    import oracle
    per, _ = ctx.reduce(tasks, sc.BATCHED)
    bad = []
    for p in pids:
        x = res.x[p * res.n:(p + 1) * res.n].cpu().numpy()
        y = res.y[p * res.n:(p + 1) * res.n].cpu().numpy()
        o = oracle.run_task(oracle.FMUL, oracle.SUM | oracle.MAX, res.n, x, y, c=0.1)
        if abs(per[p].sum - o.sum) > 1e-6 * abs(o.sum) or \
                np.float32(per[p].max) != np.float32(o.max):
            bad.append(p)
    return bad


def cpu_baseline(res: Resident, reps: int = 3) -> dict:
    """The oracle as it stands (single-threaded per partition), run on all 64
    partitions partition-parallel over the host's cores (one thread per core,
    each calling the unchanged oracle on distinct partitions)."""
    import oracle
    xs = [res.x[p * res.n:(p + 1) * res.n].cpu().numpy() for p in range(res.parts)]
    ys = [res.y[p * res.n:(p + 1) * res.n].cpu().numpy() for p in range(res.parts)]
    cores = max(1, min(os.cpu_count() or 1, 16, res.parts))
    oracle.lib()

    def run(idx):
        for p in idx:
            oracle.run_task(oracle.FMUL, oracle.SUM | oracle.MAX, res.n, xs[p], ys[p], c=0.1)

    times = []
    for _ in range(reps):
        ths = [threading.Thread(target=run, args=(list(range(k, res.parts, cores)),))
               for k in range(cores)]
        t0 = time.perf_counter()
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        times.append(time.perf_counter() - t0)
    t1 = time.perf_counter()
    run([0, 1])
    single = 2 * res.n / (time.perf_counter() - t1)
    med = statistics.median(times)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"value": res.parts * res.n / med, "unit": "elements/s", "cores": cores,
            "kind": "oracle", "host_cpus": os.cpu_count(), "cpu_model": model,
            "sample": f"all {res.parts} partitions x {res.n} pairs, partition-parallel over "
                      f"{cores} threads, median of {reps}",
            "single_thread_elements_per_s": single}


# ---- extras -----------------------------------------------------------------

def read_ceiling(sc, res: Resident, reps: int = 20) -> dict:
    """The measured HBM read-stream ceiling: a plain kernel that only reads
    the RDD's x and y (nontemporal float4 loads, grid-stride), timed with HIP
    events at 1, 2 and 4 blocks per CU; the best rate is the ceiling."""
    import torch
    lib = probe_lib(sc)
    fn = lib.sparkcl_probe_read2
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                   ctypes.c_void_p, ctypes.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(4 * cus, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for per_cu in (1, 2, 4):
        grid = per_cu * cus
        # whole passes only (4 quads of 4 floats per thread and array): all of
        # the RDD when the CU count divides it, as on MI355X's 256 CUs
        per_pass = 4 * 4 * 256 * grid
        n = (res.parts * res.n) // per_pass * per_pass

        def launch():
            rc = fn(res.x.data_ptr(), res.y.data_ptr(), n, grid, sink.data_ptr(),
                    stream.cuda_stream)
            if rc != 0:
                raise RuntimeError(f"sparkcl_probe_read2 failed ({rc})")
        for _ in range(3):
            launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            launch()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{per_cu}_per_cu"] = {"ms": ms, "GBps": 8 * n / (ms / 1e3) / 1e9,
                                   "bytes_per_launch": 8 * n}
    best = max(v["GBps"] for v in out.values())
    return {"GBps": best, "frac_of_peak": best / HBM_PEAK_GBS, "kernel": "k_read_ceiling",
            "grids": out}


def bench_single_partition(ctx, sc, reps=50) -> dict:
    import torch

    import datagen
    p = datagen.single_partition()[0]
    x = torch.from_numpy(p.x).cuda()
    tasks = [sc.task(sc.POLY, p.n, x, ops=sc.SUM, coef=p.coef)]
    out = {}
    dres = torch.empty(64, dtype=torch.uint8, device="cuda")
    for name, mode in (("per_launch", sc.PER_LAUNCH), ("batched", sc.BATCHED)):
        wall, ev = time_async(ctx, sc, tasks, mode, reps, 5, dres, None)
        t0 = time.perf_counter()
        for _ in range(10):
            ctx.reduce(tasks, mode)
        blocking = (time.perf_counter() - t0) / 10 * 1e6
        out[name] = {"us_per_launch": ev * 1e3, "elements_per_s": p.n / (ev / 1e3),
                     "us_blocking_call": blocking}
    out["note"] = "4 MiB fits in cache: launch-latency bound; HBM % not meaningful"
    return out


def probe_lib(sc):
    return ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(sc.__file__)),
                                    "libsparkcl_probe.so"))


def valu_ceiling(sc, pairs: int, reps: int = 3) -> dict:
    """The measured VALU ceiling of the Monte-Carlo loop: the probe kernel
    that runs the same Philox4x32-10 + quarter-disc loop body from registers
    only (no tiles, no queue, no memory), 8 blocks per CU, over the same
    number of Philox blocks.  Its clock marks give the shader clock the loop
    ran at."""
    import torch
    lib = probe_lib(sc)
    fn = lib.sparkcl_probe_valu
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rates = lib.sparkcl_probe_clock_rates
    rates.restype = ctypes.c_int
    peak_khz, wall_khz = ctypes.c_uint32(), ctypes.c_uint32()
    if rates(0, ctypes.byref(peak_khz), ctypes.byref(wall_khz)) != 0:
        raise RuntimeError("sparkcl_probe_clock_rates failed")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    per_cu = 8
    grid = per_cu * cus
    iters = max(1, pairs // (grid * 256))
    sink = torch.empty(grid * 256, dtype=torch.int32, device="cuda")
    clk = torch.zeros(4, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def launch():
        if fn(0, grid, iters, 0, 0, sink.data_ptr(), clk.data_ptr(), stream.cuda_stream) != 0:
            raise RuntimeError("sparkcl_probe_valu failed")
    launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    c = clk.cpu().tolist()
    sclk_ghz = (c[2] - c[0]) / (c[3] - c[1]) * wall_khz.value / 1e6 if c[3] > c[1] else None
    blocks = grid * 256 * iters
    return {"kernel": "k_valu (Philox loop, registers only)", "blocks_per_cu": per_cu,
            "ms": ms, "philox_blocks_per_s": blocks / (ms / 1e3),
            "shader_clock_GHz": sclk_ghz, "peak_clock_GHz": peak_khz.value / 1e6}


VALU_MIXES = {0: "philox loop", 1: "two philox blocks per iteration", 2: "v_bitop3_b32",
              3: "v_mad_u64_u32", 4: "v_add_u32", 5: "v_mul_hi_u32",
              6: "v_bitop3_b32 + v_add_u32", 7: "v_mad_u64_u32 + v_add_u32"}


def valu_probe_sweep(sc, target_ms: float = 3.0) -> list:
    """Every VALU probe mix at 1, 2, 4 and 8 blocks per CU: wave-instructions
    issued per CU per shader clock (VALU instructions per loop iteration from
    the probe library's own assembly, in probe_isa.json; the clock from the
    probe's clock marks)."""
    import torch
    lib = probe_lib(sc)
    fn = lib.sparkcl_probe_valu
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rates = lib.sparkcl_probe_clock_rates
    peak_khz, wall_khz = ctypes.c_uint32(), ctypes.c_uint32()
    if rates(0, ctypes.byref(peak_khz), ctypes.byref(wall_khz)) != 0:
        raise RuntimeError("sparkcl_probe_clock_rates failed")
    with open(os.path.join(os.path.dirname(os.path.abspath(sc.__file__)), "probe_isa.json")) as f:
        loop_valu = {int(k): v for k, v in json.load(f)["valu_per_iteration"].items()}
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(8 * cus * 256, dtype=torch.int32, device="cuda")
    clk = torch.zeros(4, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    out = []
    for mix, name in VALU_MIXES.items():
        for per_cu in (1, 2, 4, 8):
            grid = per_cu * cus
            waves = grid * 4
            iters = max(1, int(target_ms * 1e-3 * 2.4e9 * cus / (waves * loop_valu[mix])))
            ms = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                if fn(mix, grid, iters, 0, 0, sink.data_ptr(), clk.data_ptr(), stream.cuda_stream):
                    raise RuntimeError("sparkcl_probe_valu failed")
                e1.record(stream)
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            c = clk.cpu().tolist()
            ghz = (c[2] - c[0]) / (c[3] - c[1]) * wall_khz.value / 1e6
            t = sorted(ms)[1] / 1e3
            winstr = loop_valu[mix] * iters * waves
            out.append({"mix": mix, "instructions": name, "blocks_per_cu": per_cu, "ms": t * 1e3,
                        "shader_clock_GHz": ghz,
                        "wave_instr_per_cu_per_clock": winstr / cus / (t * ghz * 1e9)})
    return out


def alu_issue_peak(isa: dict) -> dict:
    """The Philox loop's VALU issue bound from the chip's unit counts and
    clock.  Each of a CU's 4 SIMDs issues one wave64 VALU instruction per 4
    clocks, or two when both can pair.  Measured on MI355X with the probe
    kernels: v_mad_u64_u32 never pairs, v_bitop3_b32 pairs with a simple
    32-bit instruction but not with another v_bitop3_b32, simple 32-bit
    instructions pair with each other.  Taking every other instruction as
    pairable gives an upper bound on the loop's rate: per 64 Philox blocks
    (one wave iteration) a SIMD needs at least
    mad + max(bitop3, (valu - mad) / 2) issue slots of 4 clocks."""
    lp = isa["philox_loop"]
    valu, mad, x3 = lp["valu"], lp["mad_u64_u32"], lp["xor3"]
    slots = mad + max(x3, (valu - mad) / 2)
    blocks_per_s = CUS * 4 * 64 * CLOCK_GHZ * 1e9 / (4 * slots)
    return {"valu_per_block": valu, "mad_u64_u32": mad, "bitop3": x3,
            "issue_slots_per_wave_iteration": slots, "philox_blocks_per_s": blocks_per_s,
            "lane_instr_per_s_T": blocks_per_s * valu / 1e12,
            "single_issue_lane_instr_per_s_T": ALU_PEAK_TOPS}


def bench_monte_carlo(ctx, sc, steps=5) -> dict:
    import torch

    import datagen
    parts = datagen.monte_carlo()
    tasks = [sc.task(sc.MC_PI, p.n, pid=p.pid) for p in parts]
    dres = torch.empty(64 * len(tasks), dtype=torch.uint8, device="cuda")
    samples = sum(p.n for p in parts)
    blocks = samples // 2
    # The shader clock ramps up over the first tens of milliseconds of
    # sustained VALU load (the register-only loop below read 3.17 ms right
    # after the batch's warm-up and 2.84 ms a few launches later), so the
    # batch is warmed up with ten launches, then the batch and the
    # register-only loop take turns twice: the batch's time is the median of
    # its two timed runs, the ceiling the faster of the loop's two.
    tasks = sc.task_array(tasks)
    time_async(ctx, sc, tasks, sc.BATCHED, 10, 0, dres, None)
    runs, ceils = [], []
    for _ in range(2):
        runs.append(time_async(ctx, sc, tasks, sc.BATCHED, steps, 1, dres, None))
        ceils.append(valu_ceiling(sc, blocks))
    wall = statistics.median(r[0] for r in runs)
    ev = statistics.median(r[1] for r in runs)
    out = {"ms": ev, "samples_per_s": samples / (ev / 1e3),
           "philox_blocks_per_s": blocks / (ev / 1e3), "samples": samples}
    # ALU roofline: VALU instructions per Philox block (one block = two
    # samples per lane) counted in the library's compiled gfx950 assembly, times
    # blocks/s, against the loop's issue bound at 256 CUs x 4 SIMDs x 2.4 GHz
    # (dual issue where the instructions can pair), and against the measured
    # ceiling of the same loop run from registers alone.
    isa = load_isa()
    ceil = max(ceils, key=lambda c: c["philox_blocks_per_s"])
    out["valu_ceiling"] = dict(ceil, runs_ms=[c["ms"] for c in ceils])
    out["launch"] = ctx.last_launch_shape()
    out["blocks_per_cu_mc_only"] = ctx.get_tuning().blocks_per_cu_mc_only
    out["runs_ms"] = [r[1] for r in runs]
    if isa and "philox_loop" in isa:
        model = alu_issue_peak(isa)
        valu = isa["philox_loop"]["valu"]
        achieved = blocks * valu / (ev / 1e3) / 1e12
        measured = ceil["philox_blocks_per_s"] * valu / 1e12
        out["roofline"] = {"bound": "alu", "achieved": achieved,
                           "peak": model["lane_instr_per_s_T"],
                           "unit": "T VALU lane-instr/s", "frac": achieved / model["lane_instr_per_s_T"],
                           "measured_ceiling": measured,
                           "frac_of_measured_ceiling": achieved / measured,
                           "issue_model": model}
    return out


def bench_array_reduce(ctx, sc, res, reps=20) -> dict:
    """Array-valued ReduceCL (vector add along the fixed tree) over the
    resident x tensor viewed as RDD elements: 64 arrays of 2^22 floats and
    65536 arrays of 4096 floats (the same 1 GiB).  HBM-bound: 4 B read per
    element plus the 4 B per column written."""
    import torch
    out = {}
    for name, (k, length) in (("64x2p22", (64, 1 << 22)), ("65536x4096", (65536, 4096))):
        rows = res.x.view(k, length)
        o = torch.empty(length, dtype=torch.float32, device="cuda")
        s = torch.cuda.current_stream()
        for _ in range(3):
            ctx.reduce_rows(rows, o, sc.VADD, stream=s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            ctx.reduce_rows(rows, o, sc.VADD, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        algo = 4 * k * length + 4 * length
        gbs = algo / (ms / 1e3) / 1e9
        out[name] = {"us": ms * 1e3, "elements_per_s": k * length / (ms / 1e3),
                     "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    return out


def bench_host_input(ctx, sc, res, reps=3) -> dict:
    """Host-resident partitions: the 64 x 2^22 FMUL RDD in pinned host memory,
    streamed through the staging ring (PCIe-inclusive), against a plain
    host-to-device copy of the same 2 GiB (the PCIe ceiling)."""
    import torch
    n, parts = res.n, res.parts
    hx, hy = res.pinned()
    tasks = [sc.task(sc.FMUL, n, hx[p * n:(p + 1) * n], hy[p * n:(p + 1) * n],
                     ops=sc.SUM | sc.MAX, c=0.1, host=True) for p in range(parts)]
    s = torch.cuda.current_stream()
    dres = torch.empty(64 * parts, dtype=torch.uint8, device="cuda")
    for _ in range(2):  # warm-up: plan, staging slots, first touch of the pinned pages
        ctx.reduce_async(tasks, sc.PER_LAUNCH, dres, stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ctx.reduce_async(tasks, sc.PER_LAUNCH, dres, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    dx = torch.empty_like(res.x)
    e0.record(s)
    for _ in range(reps):
        dx.copy_(hx, non_blocking=True)
        dx.copy_(hy, non_blocking=True)
    e1.record(s)
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / reps
    nbytes = 8 * parts * n
    del dx
    return {"ms": ms, "elements_per_s": parts * n / (ms / 1e3),
            "pcie_GBps": nbytes / (ms / 1e3) / 1e9,
            "copy_only_ms": copy_ms, "copy_only_GBps": nbytes / (copy_ms / 1e3) / 1e9,
            "frac_of_copy": copy_ms / ms}


def bench_misaligned(ctx, sc, res, dres, dtot, steps) -> dict:
    """The 64 x 2^22 FMUL RDD with every y partition shifted one element (4
    bytes) off x's 16-byte alignment: y's quads are then read at 4-byte
    alignment."""
    import torch
    y2 = torch.empty(res.parts * res.n + 4, dtype=torch.float32, device="cuda")
    y2[1:1 + res.parts * res.n].copy_(res.y)
    n = res.n
    tasks = [sc.task(sc.FMUL, n, res.x[p * n:(p + 1) * n], y2[1 + p * n:1 + (p + 1) * n],
                     ops=sc.SUM | sc.MAX, c=0.1) for p in range(res.parts)]
    w, e = time_async(ctx, sc, tasks, sc.BATCHED, steps, 2, dres, dtot)
    del y2
    return {"ms": e, "wall_ms": w, "hbm_GBps": 8 * res.parts * n / (e / 1e3) / 1e9}


def bench_chain(ctx, sc, res, reps=5) -> dict:
    """Fused map chain (sec. 3.1.3): the 64 x 2^22 FMUL RDD, then two POLY
    stages, reduced (SUM+MAX) in one pass with nothing materialised.  Unfused,
    the same chain is three passes (x,y -> z, z -> w, w -> reduce: 24 B per
    element against the fused pass's 8).  Kernel time of the blocking call
    (its own events), median of `reps`."""
    import statistics
    tasks = [sc.task(sc.FMUL, res.n, res.x[p * res.n:(p + 1) * res.n],
                     res.y[p * res.n:(p + 1) * res.n], ops=sc.SUM | sc.MAX, c=0.1)
             for p in range(res.parts)]
    stages = [sc.stage((0.5, -0.25, 0.125)), sc.stage((1.0, 2.0))]
    ctx.reduce_chain(tasks, stages)
    ms = []
    for _ in range(reps):
        ctx.reduce_chain(tasks, stages)
        ms.append(ctx.last_kernel_ms())
    k = statistics.median(ms)
    elems = res.parts * res.n
    return {"kernel_ms": k, "stages": "FMUL -> POLY2 -> POLY1", "elements_per_s": elems / (k / 1e3),
            "hbm_GBps": 8 * elems / (k / 1e3) / 1e9,
            "frac_of_hbm_peak": 8 * elems / (k / 1e3) / 1e9 / HBM_PEAK_GBS,
            "unfused_bytes_per_element": 24, "fused_bytes_per_element": 8}


def bench_wordcount(ctx, sc, reps=5) -> dict:
    """WordCount (sec. 3.2.3) over 1 GiB of device text: a 64 MiB Zipf corpus
    (vocabulary 10^5, s = 1, ending in a newline) repeated 16 times.  Checked
    against the oracle on the 64 MiB base (every count times 16); the oracle's
    single-thread rate on the base is the CPU baseline."""
    import numpy as np
    import torch

    import datagen
    import oracle
    base_n, rep = 64 << 20, 16
    base = datagen.corpus(base_n - 1, vocab=100_000)
    base = np.concatenate([base, np.frombuffer(b"\n", dtype=np.uint8)])
    text = torch.from_numpy(base).cuda().repeat(rep)
    cap = 1 << 20
    keys = torch.empty(cap, dtype=torch.int64, device="cuda")
    counts = torch.empty(cap, dtype=torch.int64, device="cuda")
    # a context of its own: its arena holds the counting table and the
    # spill regions (about 0.7 bytes per text byte)
    wctx = sc.Context(device=0, arena_bytes=2 << 30)
    wctx.wordcount(text, cap, keys, counts)          # warm-up
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, nd, nw = wctx.wordcount(text, cap, keys, counts)
        times.append(time.perf_counter() - t0)
    # the first occurrence of every distinct key (sparkcl_wordcount_locate)
    loc_times = []
    for _ in range(3):
        t0 = time.perf_counter()
        offs = wctx.wordcount_locate(text, keys, nd)
        loc_times.append(time.perf_counter() - t0)
    wctx.destroy()
    loc_sec = sorted(loc_times)[len(loc_times) // 2]
    sec = sorted(times)[len(times) // 2]
    t0 = time.perf_counter()
    ok, oc, on = oracle.wordcount(base)
    cpu_sec = time.perf_counter() - t0
    k = keys[:nd].cpu().numpy().view(np.uint64)
    c = counts[:nd].cpu().numpy().view(np.uint64)
    order = np.argsort(k)
    exact = bool(nw == rep * on and np.array_equal(k[order], ok) and
                 np.array_equal(c[order], oc * np.uint64(rep)))
    # every key's first word lies in the first copy of the base
    o = offs[:nd].cpu().numpy().view(np.uint64)
    loc_exact = bool(np.array_equal(o, oracle.wordcount_first(base, k)))
    nbytes = base_n * rep
    return {"ms": sec * 1e3, "GBps": nbytes / sec / 1e9, "words_per_s": nw / sec,
            "hbm_frac": nbytes / sec / 1e9 / HBM_PEAK_GBS, "words": nw, "distinct": nd,
            "matches_oracle": exact, "timing": "host-observed blocking call, median of 5",
            "locate": {"ms": loc_sec * 1e3, "GBps": nbytes / loc_sec / 1e9, "keys": nd,
                       "matches_oracle": loc_exact,
                       "what": "first byte offset of each distinct key's word"},
            # the scan kernel issues about 0.5 VALU, 0.5 SALU and 0.06 LDS
            # wave-instructions per text byte and inserts into an LDS hash
            # table: it is bound by instruction issue and LDS latency, not
            # by HBM (counters in the WordCount profile summary)
            "bound": {"kind": "issue (VALU, SALU, LDS table inserts)",
                      "hbm_frac": nbytes / sec / 1e9 / HBM_PEAK_GBS,
                      "summary": "profiles/k_wordcount_1gib_counters.md"},
            "cpu_baseline": {"GBps": base_n / cpu_sec / 1e9, "cores": 1, "kind": "oracle",
                             "sample": "the 64 MiB base corpus, one thread"}}


def bench_selective(ctx, sc, cpu: dict | None) -> dict:
    """Selective execution: the offload break-even (bytes) against host paths
    of a few rates, from the GPU's measured fixed offload cost and streaming
    rate; the oracle's own FMUL rates (8 B per element) when timed."""
    rates = {"host_1GBps": 1e9, "host_10GBps": 1e10}
    if cpu:
        rates["oracle_1_thread"] = 8 * cpu["single_thread_elements_per_s"]
        rates[f"oracle_{cpu['cores']}_threads"] = 8 * cpu["value"]
    out = {}
    try:
        for name, r in rates.items():
            out[name] = {"host_bytes_per_s": r, "breakeven_bytes": ctx.offload_breakeven(r)}
    except sc.SparkclError as e:  # needs 256 MiB of free arena
        out["error"] = str(e)
    return out


def bench_uneven(ctx, sc, steps=20, ceiling_gbps: float | None = None) -> dict:
    import torch

    import datagen
    sizes, kids = datagen.uneven_sizes()
    # inputs: one resident pool per input; partition p reads its own slice,
    # which starts 256-byte aligned as a separately allocated partition would
    def up(v):
        return (v + 63) // 64 * 64
    nx = sum(up(int(n)) for n, k in zip(sizes, kids) if k != datagen.MC_PI)
    ny = sum(up(int(n)) for n, k in zip(sizes, kids) if k == datagen.FMUL)
    x = torch.empty(nx, dtype=torch.float32, device="cuda")
    y = torch.empty(max(ny, 1), dtype=torch.float32, device="cuda")
    tasks, ox, oy, bytes_, elems, mc = [], 0, 0, 0, 0, 0
    for p, (n, k) in enumerate(zip(map(int, sizes), map(int, kids))):
        if k == datagen.MC_PI:
            tasks.append(sc.task(k, n, pid=p))
            mc += n
            continue
        xs = x[ox:ox + n]
        xs.copy_(torch.from_numpy(datagen.x_for(k, n, 0, p)))
        ox += up(n)
        ys = None
        if k == datagen.FMUL:
            ys = y[oy:oy + n]
            ys.copy_(torch.from_numpy(datagen.y_for(k, n, 0, p)))
            oy += up(n)
        tasks.append(sc.task(k, n, xs, ys, coef=datagen.POLY_COEF if k == 1 else (),
                             c=datagen.FMUL_C))
        bytes_ += n * (4 if k == datagen.POLY else 8)
        elems += n
    dres = torch.empty(64 * len(tasks), dtype=torch.uint8, device="cuda")
    out = {"partitions": len(tasks), "elements": int(sizes.sum()),
           "hbm_bytes": bytes_, "mc_samples": mc}
    # Steady state: after about 30 ms of each form untimed, the direct and
    # graph-replayed launches are timed in turns, three rounds of `steps`
    # launches each, and each form reports its median round.  (Timed first
    # and cold, whichever form came first in a process ran 10-15% slower
    # while the clock settled under the sustained load.)
    tasks = sc.task_array(tasks)
    for mode in (sc.BATCHED, sc.GRAPH):
        time_async(ctx, sc, tasks, mode, 60, 3, dres, None)
    rounds = {"batched": [], "graph": []}
    shapes = {}
    for _ in range(3):
        for name, mode in (("batched", sc.BATCHED), ("graph", sc.GRAPH)):
            wall, ev = time_async(ctx, sc, tasks, mode, steps, 1, dres, None)
            rounds[name].append((ev, wall))
            shapes[name] = ctx.last_launch_shape()
    for name, r in rounds.items():
        ev, wall = sorted(r)[len(r) // 2]
        out[name] = {"ms": ev, "wall_ms": wall, "rounds_ms": [v for v, _ in r],
                     "elements_per_s": int(sizes.sum()) / (ev / 1e3),
                     "launch": shapes[name]}
    wall, ev = time_async(ctx, sc, tasks, sc.PER_LAUNCH, steps, 3, dres, None)
    out["per_launch"] = {"ms": ev, "wall_ms": wall,
                         "elements_per_s": int(sizes.sum()) / (ev / 1e3),
                         "launch": ctx.last_launch_shape()}
    # the tuned entries this batch is cut and launched with (a mixed batch:
    # the mixed-batch tiles, occupancy and block size)
    t = ctx.get_tuning()
    out["tuning"] = {"tile_many": list(t.tile_many), "blocks_per_cu_many": t.blocks_per_cu_many,
                     "many_tiles_per_cu": list(t.many_tiles_per_cu),
                     "block_many": t.block_many, "blocks_per_cu": list(t.blocks_per_cu),
                     "unroll": list(t.unroll)}
    out["batched_speedup"] = out["per_launch"]["ms"] / out["batched"]["ms"]
    # lower bound: the larger of the HBM time of the POLY/FMUL bytes and the
    # VALU time of the Monte-Carlo samples (Philox blocks at the loop's issue
    # bound)
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9) * 1e3
    isa = load_isa()
    if isa and "philox_loop" in isa:
        t_valu = (mc / 2) / alu_issue_peak(isa)["philox_blocks_per_s"] * 1e3
        bound = max(t_hbm, t_valu)
        # fractions of the bound reached by the graph replay (the batch's
        # hipGraph-captured form) and by the direct launches
        lb = {"hbm_ms": t_hbm, "mc_valu_ms": t_valu, "ms": bound}
        for name in ("graph", "batched"):
            lb[f"hbm_frac_{name}"] = t_hbm / out[name]["ms"]
            lb[f"bound_frac_{name}"] = bound / out[name]["ms"]
        if ceiling_gbps:
            # the same bound with the HBM time at the measured read ceiling
            t_ceil = bytes_ / (ceiling_gbps * 1e9) * 1e3
            b2 = max(t_ceil, t_valu)
            lb.update({"hbm_ms_at_read_ceiling": t_ceil, "ms_at_read_ceiling": b2})
            for name in ("graph", "batched"):
                lb[f"bound_frac_at_read_ceiling_{name}"] = b2 / out[name]["ms"]
        out["lower_bound"] = lb
    return out


def trace_tasks(sc, tr, xp: int, yp: int, host: bool = False):
    """The serving trace as a contiguous array of sparkcl_task (filled column
    by column; a numpy record type with the C struct's layout).  host: x and
    y are pinned host arrays, and the POLY / FMUL tasks read them from there
    (SPARKCL_TASK_HOST_INPUT)."""
    import numpy as np

    import datagen
    dt = np.dtype([("kernel_id", "<u4"), ("reduce_ops", "<u4"), ("n", "<u8"), ("in0", "<u8"),
                   ("in1", "<u8"), ("out", "<u8"), ("seed", "<u8"), ("partition_id", "<u4"),
                   ("degree", "<u4"), ("coef", "<f4", (8,)), ("c", "<f4"), ("flags", "<u4")])
    assert dt.itemsize == ctypes.sizeof(sc.Task)
    assert all(dt.fields[f][1] == getattr(sc.Task, f).offset for f in dt.names)
    count = len(tr.sizes)
    a = np.zeros(count, dtype=dt)
    kid = tr.kids.astype(np.uint32)
    mc, fm, po = kid == datagen.MC_PI, kid == datagen.FMUL, kid == datagen.POLY
    a["kernel_id"] = kid
    a["reduce_ops"] = np.where(mc, sc.COUNT, sc.SUM | sc.MAX)
    a["n"] = tr.sizes
    off = tr.offsets.astype(np.uint64) * np.uint64(4)
    a["in0"] = np.where(mc, np.uint64(0), np.uint64(xp) + off)
    a["in1"] = np.where(fm, np.uint64(yp) + off, np.uint64(0))
    a["partition_id"] = np.where(mc, np.arange(count, dtype=np.uint32), 0)
    a["degree"] = np.where(po, len(datagen.POLY_COEF) - 1, 0)
    a["coef"][po, :len(datagen.POLY_COEF)] = datagen.POLY_COEF
    a["c"] = datagen.FMUL_C
    if host:
        a["flags"] = np.where(mc, 0, sc.TASK_HOST_INPUT)
    return a


def serve_run(sc, res: Resident, seconds: float, warm: float, per_task: bool,
              rate: float = 20000.0, host: bool = False, budget: int = 64 << 30) -> dict:
    """Open-loop Poisson stream, replayed by the native load generator
    (submit at the scheduled arrival times, poll for completions); latency =
    the server's completion stamp - scheduled arrival (no coordinated
    omission: a late submit counts against the server).  host: the tasks'
    inputs are in pinned host memory, so each latency includes its PCIe
    transfer.  budget: the admission budget in bytes."""
    import numpy as np

    import datagen
    count = int((seconds + warm) * rate)
    pool = res.parts * res.n
    tr = datagen.serving_trace(count, rate=rate, pool=pool)
    if host:
        hx, hy = res.pinned()
        tasks = trace_tasks(sc, tr, hx.data_ptr(), hy.data_ptr(), host=True)
    else:
        tasks = trace_tasks(sc, tr, res.x.data_ptr(), res.y.data_ptr())
    sched = np.ascontiguousarray((tr.t_arrive * 1e9).astype(np.int64))
    done = np.zeros(count, np.int64)
    status = np.zeros(count, np.int32)
    lg = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(sc.__file__)),
                                  "libsparkcl_loadgen.so"))
    run = lg.sparkcl_loadgen_run
    run.restype = ctypes.c_int
    run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                    ctypes.c_int64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64),
                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    ctx = sc.Context(device=0, arena_bytes=(4 << 30) if host else (1 << 30),
                     budget_bytes=budget, flags=sc.FLAG_SERVE_PER_TASK if per_task else 0)
    t0 = ctypes.c_int64()
    rc = run(ctx._h, tasks.ctypes.data, sched.ctypes.data, count, 20_000_000, 10_000,
             ctypes.byref(t0), done.ctypes.data, status.ctypes.data, None)
    stats = ctx.serve_stats()
    ctx.destroy()
    if rc != 0:
        raise RuntimeError(f"load generator failed: {sc.strerror(rc)}")
    first = int(warm * rate)
    lat = np.sort((done[first:] - (t0.value + sched[first:])) / 1e3)
    failed = int(np.count_nonzero(status))
    span = (int(done[first:].max()) - (t0.value + int(sched[first]))) / 1e9
    elems = int(tr.sizes[first:].sum())

    def pct(p):
        return float(lat[min(len(lat) - 1, int(math.ceil(p / 100 * len(lat))) - 1)])
    in_bytes = np.where(tr.kids == datagen.POLY, 4, np.where(tr.kids == datagen.FMUL, 8, 0))
    return {"offered_per_s": rate, "tasks": count - first, "failed": failed,
            "input_GBps": float((tr.sizes[first:] * in_bytes[first:]).sum()) / span / 1e9,
            "p50_us": pct(50), "p99_us": pct(99), "p999_us": pct(99.9),
            "mean_us": float(lat.mean()), "tasks_per_s": (count - first) / span,
            "elements_per_s": elems / span,
            "executor_launches": stats["executor_launches"],
            "admission_waits": stats["admission_waits"],
            "budget_peak_bytes": stats["budget_peak"]}


def serve_sweep(sc, res: Resident, rates=(20e3, 50e3, 100e3, 200e3, 400e3, 800e3, 1.6e6),
                seconds: float = 1.0, warm: float = 0.25, per_task: bool = False,
                host: bool = False, budget: int = 64 << 30) -> list:
    """A serving form at rising offered rates, up to saturation (where
    completions fall behind arrivals and the latency grows with the queue)."""
    out = []
    for r in rates:
        row = serve_run(sc, res, seconds, warm, per_task, r, host=host, budget=budget)
        out.append({k: row[k] for k in ("offered_per_s", "tasks_per_s", "p50_us", "p99_us",
                                        "p999_us", "failed", "admission_waits",
                                        "budget_peak_bytes", "input_GBps")})
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mc-only", action="store_true",
                    help="only run the Monte-Carlo partition workload (256 x 2^24 samples) "
                         "and print its line: the short program that VALU counters profile")
    ap.add_argument("--wc-only", action="store_true",
                    help="only run WordCount over 1 GiB of text and print its line")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only run the VALU probe kernels (the Philox loop and single-instruction "
                         "loops) at 1, 2, 4 and 8 blocks per CU and print their issue rates: the "
                         "short program that the dual-issue counters profile")
    ap.add_argument("--uneven-only", action="store_true",
                    help="only run the 4096-partition uneven batch (batched, graph replay, "
                         "per-partition launches) and print its line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (3 times): the "
                         "reference kernel that scales the HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the hot path is built and measured on a single "
              "MI355X; partitions would shard across GPUs as independent units (see the "
              "design notes), but no multi-GPU figure is produced.", file=sys.stderr)
        return 2

    import torch

    import paper_1505_01120_amd as sc
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": src.numel() * 4,
                          "bytes_written": dst.numel() * 4, "launches": 3}))
        return 0

    if args.wc_only:
        ctx = sc.Context(device=0, arena_bytes=1 << 30)
        line = {"workload": "WordCount, 1 GiB of Zipf text (vocabulary 10^5)",
                **bench_wordcount(ctx, sc)}
        ctx.destroy()
        print(json.dumps(line), flush=True)
        return 0
    if args.valu_probe:
        print(json.dumps({"valu_probe": valu_probe_sweep(sc)}), flush=True)
        return 0
    if args.uneven_only:
        ctx = sc.Context(device=0, arena_bytes=1 << 30)
        line = {"workload": "uneven batch: 4096 log-normal partitions, mixed kernels",
                **bench_uneven(ctx, sc)}
        ctx.destroy()
        print(json.dumps(line), flush=True)
        return 0
    if args.mc_only:
        ctx = sc.Context(device=0, arena_bytes=1 << 28)
        line = {"workload": "Monte-Carlo partitions, 256 x 2^24 Philox4x32-10 samples, batched",
                **bench_monte_carlo(ctx, sc)}
        ctx.destroy()
        print(json.dumps(line), flush=True)
        return 0

    parts, n = 64, 1 << 22
    log("generating the 64 x 2^22 RDD ...")
    res = Resident(parts, n)
    ctx = sc.Context(device=0, arena_bytes=1 << 30)
    tasks = res.tasks(sc)
    bad = spot_check(ctx, sc, res, tasks)
    if bad:
        log("parity spot check FAILED on partitions", bad)
        return 1
    dres = torch.empty(64 * parts, dtype=torch.uint8, device="cuda")
    dtot = torch.empty(64, dtype=torch.uint8, device="cuda")
    log("timing ...")
    wall_ms, ev_ms = time_async(ctx, sc, tasks, sc.BATCHED, args.steps, args.warmup, dres, dtot)
    elems = parts * n
    algo_bytes = 8 * elems
    achieved = algo_bytes / (ev_ms / 1e3) / 1e9
    traffic = load_traffic("fmul_rdd_batched")
    log("read ceiling ...")
    ceiling = read_ceiling(sc, res)
    line = {
        "metric": "mapCL+reduceCL elements/s and % peak HBM GB/s; p50/p99 task latency",
        "value": elems / (wall_ms / 1e3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 combine)",
        "data": "synthetic, seeded per partition (x~N(0,1), y~U[0,2))",
        "config": {"workload": "RDD of 64 partitions x 2^22 float32 pairs; FMUL z=x*y+0.1x; "
                               "per-partition SUM+MAX + RDD total; persistent executor, "
                               "cached plan", "partitions": parts, "elements": elems,
                   "mode": "batched"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "k_batch",
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "kernel_ms_per_launch": ev_ms,
                     "read_ceiling_GBps": ceiling["GBps"],
                     "frac_of_read_ceiling": achieved / ceiling["GBps"]},
        "read_ceiling": ceiling,
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(res)
    if not args.no_extras:
        ex = {}
        log("extras: per-launch RDD ...")
        wl, el = time_async(ctx, sc, tasks, sc.PER_LAUNCH, max(5, args.steps // 5), 2, dres, dtot)
        ex["fmul_rdd_per_launch"] = {"ms": el, "wall_ms": wl, "elements_per_s": elems / (el / 1e3),
                                     "hbm_GBps": algo_bytes / (el / 1e3) / 1e9}
        log("extras: RDD with y one element off x's alignment ...")
        ex["fmul_rdd_y_misaligned"] = bench_misaligned(ctx, sc, res, dres, dtot, args.steps)
        log("extras: graph replay RDD ...")
        wg, eg = time_async(ctx, sc, tasks, sc.GRAPH, args.steps, 2, dres, dtot)
        ex["fmul_rdd_graph"] = {"ms": eg, "wall_ms": wg, "elements_per_s": elems / (eg / 1e3),
                                "hbm_GBps": algo_bytes / (eg / 1e3) / 1e9,
                                "note": "the batched launch replayed from its cached hipGraph"}
        log("extras: single partition ...")
        ex["single_partition_poly"] = bench_single_partition(ctx, sc)
        log("extras: monte carlo ...")
        ex["monte_carlo"] = bench_monte_carlo(ctx, sc)
        log("extras: uneven batch ...")
        ex["uneven_batch"] = bench_uneven(ctx, sc, ceiling_gbps=ceiling["GBps"])
        log("extras: array-valued reduce ...")
        ex["array_reduce"] = bench_array_reduce(ctx, sc, res)
        log("extras: host-resident partitions ...")
        ex["host_input"] = bench_host_input(ctx, sc, res)
        log("extras: fused map chain ...")
        ex["map_chain"] = bench_chain(ctx, sc, res)
        log("extras: word count ...")
        ex["wordcount"] = bench_wordcount(ctx, sc)
        # the HBM-bound extras against the measured read ceiling as well
        for v in ex["array_reduce"].values():
            v["frac_of_read_ceiling"] = v["hbm_gbs"] / ceiling["GBps"]
        ex["map_chain"]["frac_of_read_ceiling"] = ex["map_chain"]["hbm_GBps"] / ceiling["GBps"]
        log("extras: selective execution ...")
        ex["selective_execution"] = bench_selective(ctx, sc, line.get("cpu_baseline"))
        if not args.no_serve:
            for name, per_task in (("resident", False), ("per_task_launch", True)):
                log(f"extras: serving ({name}) ...")
                ex.setdefault("serving", {})[name] = serve_run(
                    sc, res, args.serve_seconds, 1.0, per_task)
            log("extras: serving rate sweep ...")
            ex["serving"]["resident_rate_sweep"] = serve_sweep(sc, res)
            log("extras: serving rate sweep (per-task launches) ...")
            ex["serving"]["per_task_launch_rate_sweep"] = serve_sweep(
                sc, res, rates=(20e3, 50e3, 100e3, 200e3, 400e3), per_task=True)
            # a budget below the in-flight working set: 40 MiB holds the
            # largest task (4M FMUL elements, 32 MiB + partials) but not the
            # tasks that overlap it at these rates, so admission waits
            log("extras: serving under a 40 MiB budget ...")
            ex["serving"]["budget_bound_40MiB"] = serve_sweep(
                sc, res, rates=(100e3, 200e3, 400e3), budget=40 << 20)
            log("extras: serving host-resident inputs ...")
            ex["serving"]["resident_host_input"] = serve_run(
                sc, res, min(args.serve_seconds, 3.0), 1.0, False, host=True)
            ex["serving"]["host_input_rate_sweep"] = serve_sweep(
                sc, res, rates=(10e3, 20e3, 30e3, 40e3, 60e3), host=True)
        line["extras"] = ex
    ctx.destroy()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
