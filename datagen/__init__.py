"""Seeded synthetic inputs for the SparkCL map -> reduce workloads.

The one source of input bytes for both the oracle and the GPU path.  This
module holds none of the method's arithmetic (no map, reduction or Philox): it
only draws numbers from SplitMix64 streams named by (seed, partition id, tag)
and shapes them into the workloads below.

Tags: 1 = x, 2 = y, 3 = partition sizes, 4 = kernel ids, 5 = arrival gaps,
6 = serving sizes, 7 = serving kernel ids, 8 = serving input offsets.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdatagen.so")

WORDS, U_PM1, U_02, NORMAL, NORMAL64, U01_64 = 0, 1, 2, 3, 4, 5
_DTYPE = {WORDS: np.uint64, U_PM1: np.float32, U_02: np.float32,
          NORMAL: np.float32, NORMAL64: np.float64, U01_64: np.float64}

# Kernel ids of the registry and reduce-op bits (the boundary's numbering).
POLY, FMUL, MC_PI = 1, 2, 3
SUM, MAX, COUNT = 1, 2, 4

# The affine/polynomial map of the single-partition workload:
# y = 0.5 x^2 - 1.25 x + 3.0, coefficients lowest power first.
POLY_COEF = (3.0, -1.25, 0.5)
FMUL_C = 0.1


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared",
                               "-pthread", "-Wall", "-Wextra",
                               os.path.join(HERE, "datagen.c"), "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_lock = threading.Lock()


def _L() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build(force=False)
            L = ctypes.CDLL(LIB_PATH)
            L.datagen_fill.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
            L.datagen_fill.restype = ctypes.c_int
            L.datagen_fill_at.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
            L.datagen_fill_at.restype = ctypes.c_int
            _lib = L
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def fill(n: int, seed: int, pid: int, tag: int, dist: int,
         out: np.ndarray | None = None, first: int = 0) -> np.ndarray:
    """Draws first .. first + n - 1 of stream (seed, pid, tag) in
    distribution `dist`."""
    if out is None:
        out = np.empty(n, _DTYPE[dist])
    assert out.dtype == _DTYPE[dist] and out.flags.c_contiguous and out.size == n
    if n:
        rc = _L().datagen_fill_at(out.ctypes.data, first, n, seed, pid, tag, dist,
                                  _threads())
        if rc != 0:
            raise ValueError("datagen: bad distribution")
    return out


def x_for(kid: int, n: int, seed: int, pid: int) -> np.ndarray | None:
    """First input of a partition: U[-1,1) for POLY, N(0,1) for FMUL."""
    if kid == POLY:
        return fill(n, seed, pid, 1, U_PM1)
    if kid == FMUL:
        return fill(n, seed, pid, 1, NORMAL)
    return None


def y_for(kid: int, n: int, seed: int, pid: int) -> np.ndarray | None:
    """Second input of a partition: U[0,2) for FMUL."""
    if kid == FMUL:
        return fill(n, seed, pid, 2, U_02)
    return None


def lognormal_sizes(count: int, seed: int, tag: int, median: float, sigma: float,
                    lo: int, hi: int) -> np.ndarray:
    z = fill(count, seed, 0, tag, NORMAL64)
    return np.clip(np.rint(np.exp(math.log(median) + sigma * z)), lo, hi).astype(np.int64)


def uniform_kernel_ids(count: int, seed: int, tag: int) -> np.ndarray:
    w = fill(count, seed, 0, tag, WORDS)
    return (1 + (((w >> np.uint64(32)) * np.uint64(3)) >> np.uint64(32))).astype(np.int64)


@dataclass
class Part:
    """One partition task of a workload: kernel, reduce ops and inputs."""
    kid: int
    ops: int
    n: int
    pid: int
    seed: int = 0
    x: np.ndarray | None = None
    y: np.ndarray | None = None
    coef: tuple = ()
    c: float = FMUL_C


def default_ops(kid: int) -> int:
    return COUNT if kid == MC_PI else (SUM | MAX)


def make_part(kid: int, n: int, pid: int, seed: int = 0, ops: int | None = None,
              with_data: bool = True) -> Part:
    p = Part(kid=kid, ops=default_ops(kid) if ops is None else ops, n=n, pid=pid,
             seed=seed)
    if kid == POLY:
        p.coef = POLY_COEF
    if with_data:
        p.x = x_for(kid, n, seed, pid)
        p.y = y_for(kid, n, seed, pid)
    return p


# --- the five workloads -----------------------------------------------------

def single_partition(n: int = 1 << 20) -> list[Part]:
    """One partition of 2^20 floats U[-1,1) (seed 0), POLY map, SUM."""
    return [make_part(POLY, n, 0, ops=SUM)]


def fmul_rdd(parts: int = 64, n: int = 1 << 22, with_data: bool = True) -> list[Part]:
    """64 partitions of 2^22 pairs x~N(0,1), y~U[0,2); FMUL; SUM and MAX."""
    return [make_part(FMUL, n, p, ops=SUM | MAX, with_data=with_data)
            for p in range(parts)]


def monte_carlo(parts: int = 256, samples: int = 1 << 24) -> list[Part]:
    """256 partitions x 2^24 Philox samples each, seed 0, COUNT."""
    return [make_part(MC_PI, samples, p, ops=COUNT, with_data=False)
            for p in range(parts)]


def uneven_sizes(parts: int = 4096, median: int = 65536, lo: int = 1024,
                 hi: int = 8388608) -> tuple[np.ndarray, np.ndarray]:
    """Log-normal sizes (sigma = ln 4) and uniform kernel ids of the uneven RDD."""
    sizes = lognormal_sizes(parts, 0, 3, median, math.log(4.0), lo, hi)
    kids = uniform_kernel_ids(parts, 1, 4)
    return sizes, kids


def uneven_rdd(parts: int = 4096, with_data: bool = True, **kw) -> list[Part]:
    sizes, kids = uneven_sizes(parts, **kw)
    return [make_part(int(k), int(n), p, with_data=with_data)
            for p, (n, k) in enumerate(zip(sizes, kids))]


@dataclass
class Trace:
    """Open-loop serving trace: scheduled arrival (s), size, kernel id, offset."""
    t_arrive: np.ndarray
    sizes: np.ndarray
    kids: np.ndarray
    offsets: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))


def serving_trace(count: int, rate: float = 20000.0, median: int = 65536,
                  lo: int = 1024, hi: int = 4194304, pool: int = 0) -> Trace:
    """Poisson arrivals at `rate`/s (seed 2) with log-normal sizes (sigma ln 4).

    `pool` > 0 also draws, per task, an element offset into a resident input
    pool of that many elements, aligned down to 64 elements.
    """
    u = fill(count, 2, 0, 5, U01_64)
    gaps = -np.log(u) / rate
    t = np.cumsum(gaps)
    sizes = lognormal_sizes(count, 2, 6, median, math.log(4.0), lo, hi)
    kids = uniform_kernel_ids(count, 2, 7)
    offs = np.zeros(count, np.int64)
    if pool:
        w = fill(count, 2, 0, 8, WORDS)
        room = np.maximum(pool - sizes, 0).astype(np.uint64) + np.uint64(1)
        offs = ((w % room) // np.uint64(64) * np.uint64(64)).astype(np.int64)
    return Trace(t, sizes, kids, offs)


# --- WordCount corpus ----------------------------------------------------------

def vocabulary(size: int, seed: int = 0, max_len: int = 12) -> list[bytes]:
    """`size` synthetic words of lowercase letters, lengths uniform on
    [1, max_len] (stream tag 9) and letters uniform on a..z (tag 10, 16
    draws per word)."""
    lens = 1 + (fill(size, seed, 0, 9, WORDS) % np.uint64(max_len)).astype(np.int64)
    letters = (fill(size * 16, seed, 0, 10, WORDS) % np.uint64(26)).astype(np.uint8) + ord("a")
    letters = letters.reshape(size, 16)
    return [letters[i, :lens[i]].tobytes() for i in range(size)]


def corpus(nbytes: int, vocab: int = 100_000, zipf_s: float = 1.0, seed: int = 0,
           newline_every: int = 16, chunk_words: int = 1 << 22) -> np.ndarray:
    """A synthetic text of exactly `nbytes` bytes: words drawn from a Zipf(s)
    law over the vocabulary's ranks (uniforms from stream (seed, 1, 11)), each
    followed by a space, or by a newline with probability 1/newline_every
    (stream (seed, 1, 12)); the last word may be cut at the end.  The bytes
    do not depend on chunk_words.  Returned as a uint8 array."""
    words = vocabulary(vocab, seed)
    wlen = np.array([len(w) for w in words], dtype=np.int64)
    flat = np.frombuffer(b"".join(words), dtype=np.uint8)
    woff = np.concatenate(([0], np.cumsum(wlen)[:-1]))
    weights = np.arange(1, vocab + 1, dtype=np.float64) ** -zipf_s
    cdf = np.cumsum(weights)
    cdf /= cdf[-1]
    out = np.empty(nbytes, dtype=np.uint8)
    pos, first = 0, 0
    while pos < nbytes:
        # a token is at least 2 bytes, so this many words always suffice
        m = int(min(chunk_words, (nbytes - pos) // 2 + 1))
        u = fill(m, seed, 1, 11, U01_64, first=first)
        sep = fill(m, seed, 1, 12, WORDS, first=first)
        ranks = np.minimum(np.searchsorted(cdf, u, side="right"), vocab - 1)
        tl = wlen[ranks] + 1                       # word and its separator
        ends = np.cumsum(tl)
        starts = ends - tl
        idx = np.repeat(woff[ranks] - starts, tl) + np.arange(ends[-1])
        tok = flat[np.minimum(idx, flat.size - 1)]
        sepc = np.where(sep % np.uint64(newline_every) == 0, ord("\n"), ord(" ")).astype(np.uint8)
        tok[ends - 1] = sepc
        take = min(tok.size, nbytes - pos)
        out[pos:pos + take] = tok[:take]
        pos += take
        first += m
    return out
