"""ctypes binding of the SparkCL C ABI (include/sparkcl.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of libsparkcl.so.  PyTorch supplies device memory (the arena, inputs, outputs)
and streams.  If the library is not built this module raises on use; there is
no fallback path.

Names mirror the C entry points: ``Context.map`` is sparkcl_map (MapCL),
``Context.map_partition`` is sparkcl_map_partition (MapCLPartition),
``Context.reduce`` is sparkcl_reduce (ReduceCL), ``Context.reduce_arrays``
is sparkcl_reduce_arrays (ReduceCL over array-valued elements), ``Context.submit`` /
``Context.poll`` are the serving calls.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Iterable, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsparkcl.so")
TUNING_PATH = os.path.join(HERE, "tuning.json")

OK, EINVAL, ENOKERNEL, ETOOBIG, EAGAIN, EHIP, ETIMEDOUT, ESTOPPED, ENOMEM, ENOTFOUND = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
EDECLINED = -10
POLY, FMUL, MC_PI = 1, 2, 3
SUM, MAX, COUNT = 1, 2, 4
PER_LAUNCH, BATCHED, GRAPH = 0, 1, 2
VADD, VMAX = 1, 2
TASK_HOST_INPUT = 1
FLAG_SERVE_PER_TASK = 1
TUNE_BUCKETS, TUNE_MODES = 32, 3


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("ring_capacity", ctypes.c_uint32),
                ("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64),
                ("exec_blocks_per_cu", ctypes.c_uint32),
                ("idle_exit_ms", ctypes.c_uint32), ("watchdog_ms", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("tune_cache", ctypes.c_char_p),
                ("offload_min_bytes", ctypes.c_uint64)]


class Task(ctypes.Structure):
    _fields_ = [("kernel_id", ctypes.c_uint32), ("reduce_ops", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("in0", ctypes.c_void_p),
                ("in1", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("partition_id", ctypes.c_uint32),
                ("degree", ctypes.c_uint32), ("coef", ctypes.c_float * 8),
                ("c", ctypes.c_float), ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("sum", ctypes.c_double), ("max", ctypes.c_float),
                ("status", ctypes.c_int32), ("count", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("t_arrive_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_uint32 * 3), ("blocks_per_cu_many", ctypes.c_uint32),
                ("tile_many", ctypes.c_uint32 * 3), ("block", ctypes.c_uint32 * 3),
                ("block_many", ctypes.c_uint32), ("unroll", ctypes.c_uint32 * 3),
                ("many_tiles_per_cu", ctypes.c_uint32 * 2),
                ("blocks_per_cu_mc_only", ctypes.c_uint32),
                ("tile", ((ctypes.c_uint32 * TUNE_BUCKETS) * 3) * TUNE_MODES)]


class Stage(ctypes.Structure):
    _fields_ = [("kernel_id", ctypes.c_uint32), ("degree", ctypes.c_uint32),
                ("coef", ctypes.c_float * 8)]


def stage(coef: Sequence[float]) -> Stage:
    """A POLY chain stage with coefficients coef[k] of v^k."""
    s = Stage()
    s.kernel_id = POLY
    s.degree = max(len(coef) - 1, 0)
    for i, v in enumerate(coef):
        s.coef[i] = v
    return s


class ServeStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "submitted", "admitted", "completed", "failed", "pending", "in_flight",
        "budget_in_use", "budget_peak", "admission_waits", "executor_launches")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class LaunchShape(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in (
        "grid", "block", "ntiles", "ntasks", "tile_table", "mixed", "mode")] + \
        [("mixed_tile", ctypes.c_uint32 * 3)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["mixed_tile"] = list(self.mixed_tile)
        return d


assert ctypes.sizeof(Task) == 96 and ctypes.sizeof(Result) == 64

# Every symbol declared in include/sparkcl.h.
EXPORTS = ("sparkcl_init", "sparkcl_destroy", "sparkcl_map", "sparkcl_map_partition",
           "sparkcl_reduce", "sparkcl_reduce_async", "sparkcl_reduce_arrays",
           "sparkcl_reduce_rows", "sparkcl_reduce_chain",
           "sparkcl_submit", "sparkcl_poll",
           "sparkcl_serve_stats_get", "sparkcl_serve_drain", "sparkcl_get_tuning",
           "sparkcl_set_tuning", "sparkcl_autotune", "sparkcl_strerror",
           "sparkcl_last_error", "sparkcl_last_kernel_ms", "sparkcl_version",
           "sparkcl_offload_breakeven", "sparkcl_wordcount", "sparkcl_wordcount_locate",
           "sparkcl_reduce_noalloc",
           "sparkcl_last_launch_shape")


class SparkclError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str):
        super().__init__(f"{what}: {detail} (code {code})")
        self.code = code


_lib = None
_lock = threading.Lock()


def load() -> ctypes.CDLL:
    """Load libsparkcl.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with python -m paper_1505_01120_amd.build "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        TP, RP = ctypes.POINTER(Task), ctypes.POINTER(Result)
        sig = {
            "sparkcl_init": ([ctypes.POINTER(Config), ctypes.POINTER(P)], I32),
            "sparkcl_destroy": ([P], I32),
            "sparkcl_map": ([P, TP, U32, P], I32),
            "sparkcl_map_partition": ([P, TP, U32, I32, RP, P], I32),
            "sparkcl_reduce": ([P, TP, U32, I32, RP, RP, P], I32),
            "sparkcl_reduce_async": ([P, TP, U32, I32, P, P, P], I32),
            "sparkcl_reduce_noalloc": ([P, TP, U32, P, P, P], I32),
            "sparkcl_reduce_arrays": ([P, U32, ctypes.POINTER(P), U32, U64, P, P], I32),
            "sparkcl_reduce_rows": ([P, U32, P, U64, U32, U64, P, P], I32),
            "sparkcl_reduce_chain": ([P, TP, U32, ctypes.POINTER(Stage), U32, RP, RP, P], I32),
            "sparkcl_submit": ([P, TP, ctypes.POINTER(U64)], I32),
            "sparkcl_poll": ([P, U64, RP], I32),
            "sparkcl_serve_stats_get": ([P, ctypes.POINTER(ServeStats)], I32),
            "sparkcl_serve_drain": ([P, U32], I32),
            "sparkcl_get_tuning": ([P, ctypes.POINTER(Tuning)], I32),
            "sparkcl_set_tuning": ([P, ctypes.POINTER(Tuning)], I32),
            "sparkcl_autotune": ([P, U32, U32, ctypes.c_char_p], I32),
            "sparkcl_strerror": ([I32], ctypes.c_char_p),
            "sparkcl_last_error": ([], ctypes.c_char_p),
            "sparkcl_last_kernel_ms": ([P, ctypes.POINTER(ctypes.c_float)], I32),
            "sparkcl_last_launch_shape": ([P, ctypes.POINTER(LaunchShape)], I32),
            "sparkcl_version": ([], ctypes.c_char_p),
            "sparkcl_offload_breakeven": ([P, ctypes.c_double, ctypes.POINTER(U64)], I32),
            "sparkcl_wordcount": ([P, P, U64, P, P, U64, ctypes.POINTER(U64),
                                   ctypes.POINTER(U64), P], I32),
            "sparkcl_wordcount_locate": ([P, P, U64, P, U64, P, P], I32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
        return L


def _check(rc: int, what: str) -> int:
    if rc < 0:
        L = load()
        raise SparkclError(rc, L.sparkcl_strerror(rc).decode(),
                           f"{what}: {L.sparkcl_last_error().decode()}")
    return rc


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data  # numpy array


def task(kernel_id: int, n: int, x=None, y=None, out=None, ops: int | None = None,
         seed: int = 0, pid: int = 0, coef: Sequence[float] = (), c: float = 0.1,
         host: bool = False) -> Task:
    """A partition task; x / y / out are device tensors (or raw device
    addresses).  host=True: x / y are host arrays (CPU tensors, preferably
    pinned, numpy arrays or raw host addresses) streamed by the library."""
    t = Task()
    t.flags = TASK_HOST_INPUT if host else 0
    t.kernel_id = kernel_id
    t.reduce_ops = ops if ops is not None else (COUNT if kernel_id == MC_PI else SUM | MAX)
    t.n = n
    t.in0, t.in1, t.out = _ptr(x), _ptr(y), _ptr(out)
    t.seed, t.partition_id = seed, pid
    t.degree = max(len(coef) - 1, 0)
    for i, v in enumerate(coef):
        t.coef[i] = v
    t.c = c
    return t


class TaskArray:
    """A contiguous sparkcl_task array built once from a task list, for calls
    that replay the same batch: passing it instead of the list skips the
    per-call conversion of every task (on a 4096-task batch that conversion
    costs the host about as long as the GPU takes to run the batch)."""

    def __init__(self, tasks: Iterable[Task]):
        tasks = list(tasks)
        self.n = len(tasks)
        self.arr = (Task * max(self.n, 1))(*tasks)

    def __len__(self) -> int:
        return self.n


def task_array(tasks: Iterable[Task]) -> TaskArray:
    return TaskArray(tasks)


def _array(tasks):
    if isinstance(tasks, TaskArray):
        return tasks.arr, tasks.n
    tasks = list(tasks)
    arr = (Task * max(len(tasks), 1))(*tasks)
    return arr, len(tasks)


def _stream(stream, device: int) -> int | None:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream(device).cuda_stream


class Context:
    """A SparkCL context on one GPU, with a torch-allocated arena."""

    def __init__(self, device: int = 0, arena_bytes: int = 1 << 30, budget_bytes: int = 0,
                 ring_capacity: int = 0, flags: int = 0, tune_cache: str | None = TUNING_PATH,
                 idle_exit_ms: int = 0, watchdog_ms: int = 0, exec_blocks_per_cu: int = 0,
                 arena=None, offload_min_bytes: int = 0):
        import torch
        L = load()
        self.device = device
        self._arena = arena if arena is not None else torch.empty(
            arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        cfg = Config()
        cfg.device = device
        cfg.ring_capacity = ring_capacity
        cfg.arena = self._arena.data_ptr()
        cfg.arena_bytes = self._arena.numel() * self._arena.element_size()
        cfg.budget_bytes = budget_bytes
        cfg.exec_blocks_per_cu = exec_blocks_per_cu
        cfg.idle_exit_ms = idle_exit_ms
        cfg.watchdog_ms = watchdog_ms
        cfg.flags = flags
        self._tune = tune_cache.encode() if tune_cache and os.path.exists(tune_cache) else None
        cfg.tune_cache = self._tune
        cfg.offload_min_bytes = offload_min_bytes
        h = ctypes.c_void_p()
        _check(L.sparkcl_init(ctypes.byref(cfg), ctypes.byref(h)), "sparkcl_init")
        self._h = h

    # -- lifecycle ----------------------------------------------------------
    def destroy(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            rc = load().sparkcl_destroy(self._h)
            self._h = ctypes.c_void_p()
            _check(rc, "sparkcl_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # -- MapCL / MapCLPartition / ReduceCL ------------------------------------
    def map(self, tasks: Iterable[Task], stream=None) -> None:
        arr, n = _array(tasks)
        _check(load().sparkcl_map(self._h, arr, n, _stream(stream, self.device)), "sparkcl_map")

    def map_partition(self, tasks: Iterable[Task], mode: int = BATCHED,
                      stream=None) -> list[Result]:
        arr, n = _array(tasks)
        res = (Result * max(n, 1))()
        _check(load().sparkcl_map_partition(self._h, arr, n, mode, res,
                                            _stream(stream, self.device)),
               "sparkcl_map_partition")
        return list(res[:n])

    def reduce(self, tasks: Iterable[Task], mode: int = BATCHED,
               stream=None) -> tuple[list[Result], Result]:
        arr, n = _array(tasks)
        res = (Result * max(n, 1))()
        tot = Result()
        _check(load().sparkcl_reduce(self._h, arr, n, mode, res, ctypes.byref(tot),
                                     _stream(stream, self.device)), "sparkcl_reduce")
        return list(res[:n]), tot

    def reduce_async(self, tasks, mode: int, dev_results=None, dev_total=None,
                     stream=None) -> None:
        """Results land in device memory (uint8 tensors of 64 B per result)."""
        arr, n = _array(tasks)
        _check(load().sparkcl_reduce_async(self._h, arr, n, mode, _ptr(dev_results),
                                           _ptr(dev_total), _stream(stream, self.device)),
               "sparkcl_reduce_async")

    def reduce_noalloc(self, tasks, dev_results=None, dev_total=None, stream=None) -> None:
        """The batched reduce_async with its workspaces in the library's fixed
        device array instead of the arena (results: 64 B per result)."""
        arr, n = _array(tasks)
        _check(load().sparkcl_reduce_noalloc(self._h, arr, n, _ptr(dev_results),
                                             _ptr(dev_total), _stream(stream, self.device)),
               "sparkcl_reduce_noalloc")

    def reduce_chain(self, tasks: Iterable[Task], stages: Sequence[Stage],
                     stream=None) -> tuple[list[Result], Result]:
        """ReduceCL over fused map chains: each task's map, then `stages`."""
        arr, n = _array(tasks)
        st = (Stage * max(len(stages), 1))(*stages)
        res = (Result * max(n, 1))()
        tot = Result()
        _check(load().sparkcl_reduce_chain(self._h, arr, n, st, len(stages), res,
                                           ctypes.byref(tot), _stream(stream, self.device)),
               "sparkcl_reduce_chain")
        return list(res[:n]), tot

    def reduce_arrays(self, arrays: Sequence, out, combiner: int = VADD,
                      stream=None) -> None:
        """Array-valued ReduceCL: fold the RDD elements (device float32
        arrays of one length, in RDD order) with the combiner along the
        library's fixed tree into `out`.  Asynchronous on `stream`."""
        ptrs = [_ptr(a) for a in arrays]
        n = len(ptrs)
        table = (ctypes.c_void_p * max(n, 1))(*ptrs)
        length = int(out.numel()) if out is not None else 0
        _check(load().sparkcl_reduce_arrays(self._h, combiner, table, n, length, _ptr(out),
                                            _stream(stream, self.device)),
               "sparkcl_reduce_arrays")

    def reduce_rows(self, rows, out, combiner: int = VADD, stream=None) -> None:
        """Array-valued ReduceCL over the rows of a 2-D device tensor (each
        row one RDD element, unit inner stride) into `out`."""
        if rows.dim() != 2 or (rows.size(1) > 1 and rows.stride(1) != 1):
            raise ValueError("rows must be a 2-D tensor with contiguous rows")
        k, length = rows.shape
        _check(load().sparkcl_reduce_rows(self._h, combiner, rows.data_ptr(), rows.stride(0),
                                          k, length, _ptr(out), _stream(stream, self.device)),
               "sparkcl_reduce_rows")

    # -- serving ------------------------------------------------------------
    def submit(self, t: Task) -> int:
        ticket = ctypes.c_uint64()
        _check(load().sparkcl_submit(self._h, ctypes.byref(t), ctypes.byref(ticket)),
               "sparkcl_submit")
        return ticket.value

    def poll(self, ticket: int) -> Result | None:
        r = Result()
        rc = load().sparkcl_poll(self._h, ticket, ctypes.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc, "sparkcl_poll")
        return r

    def serve_stats(self) -> dict:
        s = ServeStats()
        _check(load().sparkcl_serve_stats_get(self._h, ctypes.byref(s)), "serve_stats")
        return s.as_dict()

    def serve_drain(self, timeout_ms: int = 10000) -> None:
        _check(load().sparkcl_serve_drain(self._h, timeout_ms), "sparkcl_serve_drain")

    # -- tuning and diagnostics ---------------------------------------------
    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(load().sparkcl_get_tuning(self._h, ctypes.byref(t)), "sparkcl_get_tuning")
        return t

    def set_tuning(self, t: Tuning) -> None:
        _check(load().sparkcl_set_tuning(self._h, ctypes.byref(t)), "sparkcl_set_tuning")

    def autotune(self, lo_log2: int = 10, hi_log2: int = 22, path: str | None = None) -> None:
        _check(load().sparkcl_autotune(self._h, lo_log2, hi_log2,
                                       path.encode() if path else None), "sparkcl_autotune")

    def wordcount(self, text, capacity: int, keys=None, counts=None, stream=None):
        """WordCount over a device uint8 tensor: (keys, counts, distinct, words),
        keys/counts as int64 device tensors of `capacity` (first `distinct`
        entries valid, unordered)."""
        import torch
        if keys is None:
            keys = torch.empty(max(capacity, 1), dtype=torch.int64, device=text.device)
        if counts is None:
            counts = torch.empty(max(capacity, 1), dtype=torch.int64, device=text.device)
        nd, nw = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().sparkcl_wordcount(self._h, _ptr(text), text.numel(), _ptr(keys),
                                        _ptr(counts), capacity, ctypes.byref(nd),
                                        ctypes.byref(nw), _stream(stream, self.device)),
               "sparkcl_wordcount")
        return keys, counts, nd.value, nw.value

    def wordcount_locate(self, text, keys, nkeys: int | None = None, offsets=None, stream=None):
        """First byte offset in `text` (device uint8 tensor) of each of the
        first `nkeys` keys of `keys` (device int64 tensor, distinct), as an
        int64 device tensor; -1 (UINT64_MAX) for a key no word has."""
        import torch
        n = keys.numel() if nkeys is None else nkeys
        if offsets is None:
            offsets = torch.empty(max(n, 1), dtype=torch.int64, device=text.device)
        _check(load().sparkcl_wordcount_locate(self._h, _ptr(text), text.numel(), _ptr(keys),
                                               n, _ptr(offsets), _stream(stream, self.device)),
               "sparkcl_wordcount_locate")
        return offsets

    def offload_breakeven(self, host_bytes_per_s: float) -> int:
        """Smallest offload cost (bytes) at which this GPU beats a host path of
        the given throughput (selective execution threshold)."""
        v = ctypes.c_uint64()
        _check(load().sparkcl_offload_breakeven(self._h, float(host_bytes_per_s), ctypes.byref(v)),
               "sparkcl_offload_breakeven")
        return v.value

    def last_kernel_ms(self) -> float:
        v = ctypes.c_float()
        _check(load().sparkcl_last_kernel_ms(self._h, ctypes.byref(v)), "last_kernel_ms")
        return v.value

    def last_launch_shape(self) -> dict:
        """Grid, block size, tile count and tile table of the last
        reduce/map_partition call."""
        v = LaunchShape()
        _check(load().sparkcl_last_launch_shape(self._h, ctypes.byref(v)), "last_launch_shape")
        return v.as_dict()


def version() -> str:
    return load().sparkcl_version().decode()


def strerror(code: int) -> str:
    return load().sparkcl_strerror(code).decode()
