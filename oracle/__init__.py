"""ctypes binding of the SparkCL map -> reduce oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the GPU product path
(``paper_1505_01120_amd``) never does, and the two share no code.

Every function here is a thin marshalling wrapper over the C oracle, which is a
single-threaded, index-ordered, FP64-summing reference of MapCL,
MapCLPartition and ReduceCL (paper sec. 3.1.3) for the three built-in kernels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

POLY, FMUL, MC_PI = 1, 2, 3
SUM, MAX, COUNT = 1, 2, 4

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (contraction off)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, os.path.join(HERE, "oracle.c"),
                               "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Task(ctypes.Structure):
    _fields_ = [("kernel_id", ctypes.c_uint32), ("reduce_ops", ctypes.c_uint32),
                ("n", ctypes.c_uint64),
                ("in0", ctypes.c_void_p), ("in1", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("partition_id", ctypes.c_uint32),
                ("degree", ctypes.c_uint32), ("coef", ctypes.c_float * 8),
                ("c", ctypes.c_float)]


class Result(ctypes.Structure):
    _fields_ = [("sum", ctypes.c_double), ("max", ctypes.c_float),
                ("pad", ctypes.c_uint32), ("count", ctypes.c_uint64),
                ("n", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {"sum": self.sum, "max": self.max, "count": self.count, "n": self.n}


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build(force=False)
            L = ctypes.CDLL(LIB_PATH)
            P = ctypes.c_void_p
            U64, U32 = ctypes.c_uint64, ctypes.c_uint32
            L.oracle_poly_map.argtypes = [P, U64, U32, P, P]
            L.oracle_fmul_map.argtypes = [P, P, U64, ctypes.c_float, P]
            L.oracle_sum.argtypes = [P, U64]
            L.oracle_sum.restype = ctypes.c_double
            L.oracle_sum_f64.argtypes = [P, U64]
            L.oracle_sum_f64.restype = ctypes.c_double
            L.oracle_max.argtypes = [P, U64]
            L.oracle_max.restype = ctypes.c_float
            L.oracle_philox4x32_10.argtypes = [P, P, P]
            L.oracle_mc_count.argtypes = [U64, U32, U64, U64]
            L.oracle_mc_count.restype = U64
            L.oracle_task_run.argtypes = [ctypes.POINTER(Task), ctypes.POINTER(Result)]
            L.oracle_task_run.restype = ctypes.c_int
            L.oracle_tree_reduce_arrays.argtypes = [U32, P, U32, U64, P]
            L.oracle_tree_reduce_arrays.restype = ctypes.c_int
            L.oracle_fnv1a64.argtypes = [P, U64]
            L.oracle_fnv1a64.restype = U64
            L.oracle_wordcount.argtypes = [P, U64, P, P, U64, ctypes.POINTER(U64),
                                           ctypes.POINTER(U64)]
            L.oracle_wordcount.restype = ctypes.c_int
            L.oracle_wordcount_first.argtypes = [P, U64, P, U64, P]
            L.oracle_wordcount_first.restype = ctypes.c_int
            L.oracle_rdd_total.argtypes = [ctypes.POINTER(Result), U64, U32,
                                           ctypes.POINTER(Result)]
            _lib = L
    return _lib


def _f32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def poly_map(x, coef) -> np.ndarray:
    """O1: y_i = Horner(coef, x_i); coef[k] multiplies x^k; degree = len(coef)-1."""
    x = _f32(x)
    c = np.zeros(8, np.float32)
    c[:len(coef)] = coef
    y = np.empty_like(x)
    lib().oracle_poly_map(_ptr(x), x.size, len(coef) - 1, c.ctypes.data, _ptr(y))
    return y


def fmul_map(x, y, c=np.float32(0.1)) -> np.ndarray:
    """O2: z_i = fl(fl(x_i*y_i) + fl(c*x_i))."""
    x, y = _f32(x), _f32(y)
    assert x.shape == y.shape
    z = np.empty_like(x)
    lib().oracle_fmul_map(_ptr(x), _ptr(y), x.size, float(np.float32(c)), _ptr(z))
    return z


def fsum(v) -> float:
    """O3: FP64 Neumaier sum of float32 values in index order."""
    v = _f32(v)
    return lib().oracle_sum(_ptr(v), v.size)


def fsum64(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().oracle_sum_f64(_ptr(v), v.size)


def fmax(v) -> np.float32:
    """O4: max in index order from -inf."""
    v = _f32(v)
    return np.float32(lib().oracle_max(_ptr(v), v.size))


def philox(ctr, key) -> np.ndarray:
    """O5: Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().oracle_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def mc_count(seed: int, pid: int, lo: int, hi: int | None = None) -> int:
    """O6: hits among samples [lo, hi) (or [0, lo) when hi is None)."""
    if hi is None:
        lo, hi = 0, lo
    return int(lib().oracle_mc_count(seed, pid, lo, hi))


def make_task(kernel_id, ops, n, x=None, y=None, *, seed=0, pid=0, coef=(),
              c=0.1) -> tuple[Task, tuple]:
    """Build an oracle Task; returns (task, keepalive) so arrays outlive it."""
    t = Task()
    t.kernel_id, t.reduce_ops, t.n = kernel_id, ops, n
    keep = []
    if x is not None:
        x = _f32(x)
        keep.append(x)
        t.in0 = _ptr(x)
    if y is not None:
        y = _f32(y)
        keep.append(y)
        t.in1 = _ptr(y)
    t.seed, t.partition_id = seed, pid
    t.degree = max(len(coef) - 1, 0)
    for i, v in enumerate(coef):
        t.coef[i] = v
    t.c = float(np.float32(c))
    return t, tuple(keep)


def run_task(kernel_id, ops, n, x=None, y=None, **kw) -> Result:
    """Oracle result of one partition task (map fused with the reductions)."""
    t, keep = make_task(kernel_id, ops, n, x, y, **kw)
    r = Result()
    rc = lib().oracle_task_run(ctypes.byref(t), ctypes.byref(r))
    del keep
    if rc != 0:
        raise ValueError("oracle: invalid task")
    return r


def rdd_total(results, ops) -> Result:
    """O7: RDD-level combine of partition results in partition order."""
    arr = (Result * len(results))(*results)
    out = Result()
    lib().oracle_rdd_total(arr, len(results), ops, ctypes.byref(out))
    return out


VADD, VMAX = 1, 2


def tree_reduce_arrays(arrays, combiner: int = VADD) -> np.ndarray:
    """O9: fold the RDD elements (a sequence of equal-length float32 arrays,
    or the rows of a 2-D array) with the combiner along the fixed tree."""
    rows = [_f32(a) for a in arrays]
    if not rows:
        raise ValueError("tree reduce of an empty RDD")
    n = rows[0].size
    if any(r.size != n for r in rows):
        raise ValueError("RDD elements differ in length")
    ptrs = (ctypes.c_void_p * len(rows))(*[_ptr(r) for r in rows])
    out = np.empty(n, dtype=np.float32)
    rc = lib().oracle_tree_reduce_arrays(combiner, ptrs, len(rows), n, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_tree_reduce_arrays rejected combiner {combiner}")
    return out


def tree_reduce_rows(rows: np.ndarray, combiner: int = VADD) -> np.ndarray:
    """O9 over the rows of a 2-D float32 array (any row stride, unit column
    stride): the same fold as tree_reduce_arrays, with the row pointers built
    by numpy instead of one Python object per row."""
    if rows.ndim != 2 or rows.dtype != np.float32 or rows.strides[1] != 4:
        raise ValueError("rows must be a 2-D float32 array with contiguous rows")
    k, n = rows.shape
    if k == 0:
        raise ValueError("tree reduce of an empty RDD")
    ptrs = (np.uint64(rows.ctypes.data) +
            np.arange(k, dtype=np.uint64) * np.uint64(rows.strides[0]))
    out = np.empty(n, dtype=np.float32)
    rc = lib().oracle_tree_reduce_arrays(combiner, ptrs.ctypes.data, k, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_tree_reduce_arrays rejected combiner {combiner}")
    return out


def fnv1a64(b: bytes) -> int:
    """O10's word key: 64-bit FNV-1a of the bytes."""
    buf = np.frombuffer(bytes(b), dtype=np.uint8)
    return int(lib().oracle_fnv1a64(_ptr(buf) if buf.size else None, buf.size))


def wordcount(text) -> tuple[np.ndarray, np.ndarray, int]:
    """O10: (keys ascending, counts, total words) of a byte string or uint8 array."""
    t = np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
        else np.ascontiguousarray(text, dtype=np.uint8)
    cap = max(1, t.size // 2 + 1)
    keys = np.empty(cap, dtype=np.uint64)
    counts = np.empty(cap, dtype=np.uint64)
    nd, nw = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().oracle_wordcount(_ptr(t) if t.size else None, t.size, _ptr(keys), _ptr(counts),
                                cap, ctypes.byref(nd), ctypes.byref(nw))
    if rc != 0:
        raise MemoryError("oracle_wordcount failed")
    return keys[:nd.value].copy(), counts[:nd.value].copy(), nw.value


def wordcount_first(text, keys) -> np.ndarray:
    """O10 words: for each query key (uint64), the byte offset of the first
    word of `text` with that key, UINT64_MAX when none has it."""
    t = np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
        else np.ascontiguousarray(text, dtype=np.uint8)
    q = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty(max(q.size, 1), dtype=np.uint64)
    rc = lib().oracle_wordcount_first(_ptr(t) if t.size else None, t.size,
                                      _ptr(q) if q.size else None, q.size, _ptr(out))
    if rc != 0:
        raise MemoryError("oracle_wordcount_first failed")
    return out[:q.size].copy()


def chain_map(x, y, kid: int, coef=(), c=np.float32(0.1), stages=()) -> np.ndarray:
    """A fused map chain by composition of O1/O2: the task's map (POLY with
    `coef`, or FMUL with `c`), then each POLY stage in `stages` (coefficient
    tuples) applied to the running values."""
    v = poly_map(x, coef) if kid == ORACLE_POLY else fmul_map(x, y, c)
    for st in stages:
        v = poly_map(v, st)
    return v


ORACLE_POLY, ORACLE_FMUL = 1, 2
