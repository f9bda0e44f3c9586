"""Pins of the oracle's reductions (ReduceCL, paper sec. 3.1.3 and 3.2.2).

Closed forms on arithmetic sequences, Python's correctly rounded math.fsum,
exact rational sums by brute force, inputs that defeat uncompensated and Kahan
summation, and numpy's max.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

U64 = 2.0 ** -53


def neumaier_bound(vals, n) -> float:
    # Neumaier: |S_hat - S| <= u|S| + O(n u^2) sum|v|; generous constants.
    s = float(np.sum(np.abs(np.asarray(vals, np.float64))))
    return 4 * U64 * abs(math.fsum(vals)) + 4 * n * U64 * U64 * s + 1e-300


def faulhaber(n: int, a: F, d: F):
    """(sum x, sum x^2) of x_i = a + i d, i = 0..n-1, in closed form."""
    s1 = n * a + d * F(n * (n - 1), 2)
    s2 = n * a * a + a * d * n * (n - 1) + d * d * F((n - 1) * n * (2 * n - 1), 6)
    return s1, s2


def test_poly_sum_closed_form_degree2(oracle):
    # x_i = i/128, i < 1024: the map 0.5x^2 - 1.25x + 3 is exact in binary32
    # and every partial sum is exact in double, so the sum is the closed form.
    n = 1024
    a, d = F(0), F(1, 128)
    x = (np.arange(n) / 128.0).astype(np.float32)
    s1, s2 = faulhaber(n, a, d)
    want = F(1, 2) * s2 - F(5, 4) * s1 + 3 * n
    r = oracle.run_task(oracle.POLY, oracle.SUM, n, x, coef=(3.0, -1.25, 0.5))
    assert F(r.sum) == want


def test_poly_sum_closed_form_degree1_large(oracle):
    # y = 0.5 i + 3 over i < 2^20: sum = n(n-1)/4 + 3n exactly.
    n = 1 << 20
    x = np.arange(n, dtype=np.float32)
    r = oracle.run_task(oracle.POLY, oracle.SUM | oracle.MAX, n, x, coef=(3.0, 0.5))
    assert F(r.sum) == F(n * (n - 1), 4) + 3 * n
    assert r.max == np.float32(0.5 * (n - 1) + 3)
    assert r.n == n


def test_fmul_sum_closed_form(oracle):
    # x = -1 + i/256, y = 0.5 + i/128, c = 0.25 (exact): sum = sum xy + c sum x.
    n = 512
    i = np.arange(n)
    x = (-1.0 + i / 256.0).astype(np.float32)
    y = (0.5 + i / 128.0).astype(np.float32)
    ax, dx, ay, dy = F(-1), F(1, 256), F(1, 2), F(1, 128)
    sx, _ = faulhaber(n, ax, dx)
    si = F(n * (n - 1), 2)
    si2 = F((n - 1) * n * (2 * n - 1), 6)
    sxy = n * ax * ay + (ax * dy + ay * dx) * si + dx * dy * si2
    r = oracle.run_task(oracle.FMUL, oracle.SUM, n, x, y, c=0.25)
    assert F(r.sum) == sxy + F(1, 4) * sx


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sum_matches_fsum(oracle, datagen, seed):
    # math.fsum is correctly rounded; Neumaier lies within its error bound.
    n = 300_000
    v = datagen.fill(n, seed, 0, 1, datagen.NORMAL)
    got = oracle.fsum(v)
    want = math.fsum(v.astype(np.float64))
    assert abs(got - want) <= neumaier_bound(v.astype(np.float64), n)


def test_sum_brute_force_fraction(oracle, datagen):
    for n in (0, 1, 2, 3, 17, 64, 255, 256):
        v = datagen.fill(n, 11, n, 1, datagen.NORMAL) * np.float32(1000)
        exact = sum((F(float(t)) for t in v), F(0))
        got = oracle.fsum(v)
        assert abs(F(got) - exact) <= F(neumaier_bound(v.astype(np.float64), n))
        if n == 0:
            assert got == 0.0 and math.copysign(1, got) == 1


@pytest.mark.parametrize("vals,exact", [
    ([2.0 ** 60, 1.0, -2.0 ** 60], 1.0),            # plain summation gives 0
    ([1.0, 2.0 ** 100, 1.0, -2.0 ** 100], 2.0),     # Kahan gives 0, Neumaier 2
    ([3.0, 2.0 ** 70, -1.0, -2.0 ** 70, 0.5], 2.5),
])
def test_sum_defeats_naive_and_kahan(oracle, vals, exact):
    v = np.asarray(vals, np.float32)
    assert oracle.fsum(v) == exact


def test_sum_f64_rdd_level(oracle):
    v = np.array([1e300, 1.0, -1e300, 2.0 ** -30], np.float64)
    assert oracle.fsum64(v) == 1.0 + 2.0 ** -30


def test_max_matches_numpy(oracle, datagen):
    for n in (1, 5, 1000, 123457):
        v = datagen.fill(n, 5, n, 1, datagen.NORMAL)
        assert oracle.fmax(v).view(np.uint32) == np.max(v).view(np.uint32)
        perm = v[datagen.fill(n, 6, n, 1, datagen.WORDS).argsort()]
        assert oracle.fmax(perm) == oracle.fmax(v)


def test_max_empty_and_task_identities(oracle):
    assert oracle.fmax(np.zeros(0, np.float32)) == -np.inf
    r = oracle.run_task(oracle.FMUL, oracle.SUM | oracle.MAX, 0,
                        np.zeros(0, np.float32), np.zeros(0, np.float32))
    assert r.sum == 0.0 and math.copysign(1, r.sum) == 1
    assert r.max == -np.inf and r.count == 0 and r.n == 0


def test_task_masks_unrequested(oracle, datagen):
    x = datagen.fill(1000, 0, 0, 1, datagen.U_PM1)
    r = oracle.run_task(oracle.POLY, oracle.MAX, 1000, x, coef=(3.0, -1.25, 0.5))
    assert r.sum == 0.0 and r.max == np.max(oracle.poly_map(x, (3.0, -1.25, 0.5)))
    r = oracle.run_task(oracle.POLY, oracle.SUM, 1000, x, coef=(3.0, -1.25, 0.5))
    assert r.max == -np.inf


def test_task_rejects_bad_requests(oracle):
    x = np.zeros(4, np.float32)
    with pytest.raises(ValueError):
        oracle.run_task(oracle.POLY, oracle.COUNT, 4, x, coef=(1.0,))
    with pytest.raises(ValueError):
        oracle.run_task(oracle.MC_PI, oracle.SUM, 4)
    with pytest.raises(ValueError):
        oracle.run_task(9, oracle.SUM, 4, x)
    with pytest.raises(ValueError):
        oracle.run_task(oracle.FMUL, 0, 4, x, x)


def test_task_equals_map_then_reduce(oracle, datagen):
    n = 100_003
    x = datagen.fill(n, 0, 3, 1, datagen.NORMAL)
    y = datagen.fill(n, 0, 3, 2, datagen.U_02)
    z = oracle.fmul_map(x, y)
    r = oracle.run_task(oracle.FMUL, oracle.SUM | oracle.MAX, n, x, y)
    assert r.sum == oracle.fsum(z) and r.max == np.max(z)
    assert abs(r.sum - math.fsum(z.astype(np.float64))) <= neumaier_bound(
        z.astype(np.float64), n)


def test_rdd_total(oracle, datagen):
    parts = []
    for p in range(7):
        n = 1000 + 37 * p
        x = datagen.fill(n, 0, p, 1, datagen.NORMAL)
        y = datagen.fill(n, 0, p, 2, datagen.U_02)
        parts.append(oracle.run_task(oracle.FMUL, oracle.SUM | oracle.MAX, n, x, y))
    tot = oracle.rdd_total(parts, oracle.SUM | oracle.MAX)
    sums = [r.sum for r in parts]
    assert abs(tot.sum - math.fsum(sums)) <= neumaier_bound(sums, len(sums))
    assert tot.max == max(r.max for r in parts)
    assert tot.n == sum(r.n for r in parts)
    mc = [oracle.run_task(oracle.MC_PI, oracle.COUNT, 100 + p, seed=0, pid=p)
          for p in range(5)]
    tm = oracle.rdd_total(mc, oracle.COUNT)
    assert tm.count == sum(r.count for r in mc) and tm.sum == 0.0


def test_rdd_total_is_compensated(oracle):
    # partition sums 2^60, 1, -2^60, 0.25: the RDD-level fold must return 1.25
    parts = []
    for s in (2.0 ** 60, 1.0, -2.0 ** 60, 0.25):
        r = oracle.Result()
        r.sum, r.max, r.count, r.n = s, np.float32(s), 0, 1
        parts.append(r)
    tot = oracle.rdd_total(parts, oracle.SUM | oracle.MAX)
    assert tot.sum == 1.25 and tot.max == np.float32(2.0 ** 60) and tot.n == 4
