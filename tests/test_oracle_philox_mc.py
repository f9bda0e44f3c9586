"""Pins of the oracle's Philox4x32-10 and Monte-Carlo count (SparkCLPi, sec. 3.2.1).

Philox is checked against two independent implementations that ship as header
source in this image (PyTorch's at::philox_engine and rocRAND's engine), both
compiled here for the CPU.  The hit count is checked by brute force: the words
come from PyTorch's engine (not the oracle) and the disc test is done with
exact rationals.
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction as F

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include() -> str:
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "include")


@pytest.fixture(scope="session")
def aten_philox(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("xcheck") / "aten_philox")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", _torch_include(),
                           os.path.join(HERE, "xcheck", "aten_philox.cpp"), "-o", exe])
    return exe


@pytest.fixture(scope="session")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("xcheck") / "rocrand_philox")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                           os.path.join(HERE, "xcheck", "rocrand_philox.cpp"),
                           "-o", exe])
    return exe


def run_helper(exe, rows):
    text = "".join("%x %x %x %x %x %x\n" % tuple(r) for r in rows)
    out = subprocess.run([exe], input=text, capture_output=True, text=True,
                         check=True).stdout.split()
    return np.array([int(w, 16) for w in out], np.uint64).reshape(-1, 4)


def oracle_rows(oracle, rows):
    return np.array([oracle.philox(r[2:], r[:2]) for r in rows], np.uint64)


def random_rows(datagen, count, seed, ctr1_bits=32):
    w = datagen.fill(3 * count, seed, 0, 9, datagen.WORDS).reshape(count, 3)
    rows = []
    for a, b, c in w:
        a, b, c = int(a), int(b), int(c)
        rows.append((a & 0xffffffff, a >> 32, b & 0xffffffff,
                     (b >> 32) & ((1 << ctr1_bits) - 1), c & 0xffffffff, c >> 32))
    return rows


def test_philox_vs_aten(oracle, datagen, aten_philox):
    rows = [(0, 0, 0, 0, 0, 0), (0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff,
                                 0xffffffff, 0xffffffff)]
    rows += random_rows(datagen, 3000, 1)
    rows += [(s & 0xffffffff, s >> 32, j, 0, p, 0)
             for s in (0, 1, 12345) for p in (0, 1, 255) for j in range(8)]
    assert np.array_equal(run_helper(aten_philox, rows), oracle_rows(oracle, rows))


def test_philox_vs_rocrand(oracle, datagen, rocrand_philox):
    rows = [(0, 0, 0, 0, 0, 0)] + random_rows(datagen, 2000, 2, ctr1_bits=29)
    assert np.array_equal(run_helper(rocrand_philox, rows), oracle_rows(oracle, rows))


def brute_count(words_by_pair, lo, hi) -> int:
    """Exact disc test on the rational point (a, b) * 2^-24."""
    hits = 0
    one = F(1)
    for s in range(lo, hi):
        r = words_by_pair[s // 2]
        wa, wb = (r[0], r[1]) if s % 2 == 0 else (r[2], r[3])
        x = F(int(wa) >> 8, 1 << 24)
        y = F(int(wb) >> 8, 1 << 24)
        hits += x * x + y * y <= one
    return hits


@pytest.mark.parametrize("seed,pid,n", [(0, 0, 4096), (0, 7, 1), (0, 255, 4095),
                                        (0xDEADBEEF12345678, 3, 1001), (1, 0, 2)])
def test_mc_count_brute_force(oracle, aten_philox, seed, pid, n):
    pairs = (n + 1) // 2
    rows = [(seed & 0xffffffff, seed >> 32, j & 0xffffffff, j >> 32, pid, 0)
            for j in range(pairs)]
    words = run_helper(aten_philox, rows)
    assert oracle.mc_count(seed, pid, n) == brute_count(words, 0, n)
    # and over an odd-started window
    if n > 3:
        assert oracle.mc_count(seed, pid, 3, n) == brute_count(words, 3, n)


def test_mc_count_additive(oracle, datagen):
    n = 50_001
    total = oracle.mc_count(0, 9, 0, n)
    cuts = datagen.fill(6, 4, 0, 1, datagen.WORDS) % np.uint64(n)
    for k in map(int, cuts):
        assert oracle.mc_count(0, 9, 0, k) + oracle.mc_count(0, 9, k, n) == total
    assert oracle.mc_count(0, 9, 5, 5) == 0


def test_mc_count_statistics(oracle):
    # count/N within 5 sigma of pi/4, for two partitions of 2^21 samples.
    n = 1 << 21
    p = math.pi / 4
    sigma = math.sqrt(p * (1 - p) / n)
    for pid in (0, 1):
        c = oracle.mc_count(0, pid, n)
        assert abs(c / n - p) < 5 * sigma
    # partitions differ (the partition id is in the counter)
    assert oracle.mc_count(0, 0, 4096) != oracle.mc_count(0, 1, 4096) or \
        oracle.mc_count(0, 0, 8192) != oracle.mc_count(0, 1, 8192)


def test_mc_boundary_only_trivial_points():
    # a^2 + b^2 = 2^48 with 0 <= a, b < 2^24 has no solution, so "<=" and "<"
    # agree: check the descent argument numerically on the 2-adic ladder.
    for k in range(0, 25):
        r = 1 << k  # a^2 + b^2 = 4^k forces a, b even down to k = 0
        sols = [(a, math.isqrt(r * r - a * a)) for a in range(0, min(r, 4096) + 1)
                if math.isqrt(r * r - a * a) ** 2 == r * r - a * a]
        assert all(a in (0, r) for a, _ in sols)
