"""Pins of the oracle's elementwise maps (MapCL, paper sec. 3.1.3; Fig 3 body).

Each case is chosen so a plausible slip in oracle.c fails it: a reversed or
shifted coefficient, a dropped term, a wrong operand, a contracted multiply-add
or a skipped element.
"""
from fractions import Fraction as F

import numpy as np
import pytest


def frac32(v) -> F:
    return F(float(np.float32(v)))


def test_poly_degree2_exact_dyadic_closed_form(oracle):
    # x = k/64 on [-1, 1]: every Horner step of 0.5x^2 - 1.25x + 3 is exact in
    # binary32, so the map equals the rational polynomial bit for bit.
    ks = np.arange(-64, 65)
    x = (ks / 64.0).astype(np.float32)
    y = oracle.poly_map(x, (3.0, -1.25, 0.5))
    for xi, yi in zip(x, y):
        q = F(1, 2) * frac32(xi) ** 2 - F(5, 4) * frac32(xi) + 3
        assert frac32(yi) == q


def test_poly_degree1_integers(oracle):
    # y = 0.5 x + 3 on x = 0..2^20-1: exact; pins coefficient order (3x + 0.5
    # would differ) and that every element is written.
    x = np.arange(1 << 20, dtype=np.float32)
    y = oracle.poly_map(x, (3.0, 0.5))
    assert np.array_equal(y.astype(np.float64), 0.5 * x.astype(np.float64) + 3.0)


def test_poly_degree7_dyadic(oracle):
    # Small dyadic coefficients and x = k/4 for |k| <= 4: every step is exact.
    coef = (0.5, -0.25, 0.125, 1.0, -0.5, 0.25, -0.125, 0.0625)
    x = (np.arange(-4, 5) / 4.0).astype(np.float32)
    y = oracle.poly_map(x, coef)
    for xi, yi in zip(x, y):
        q = sum(F(c) * frac32(xi) ** k for k, c in enumerate(coef))
        assert frac32(yi) == q


def test_poly_degree0_constant(oracle):
    x = np.linspace(-5, 5, 101, dtype=np.float32)
    y = oracle.poly_map(x, (2.5,))
    assert np.all(y == np.float32(2.5))


def test_poly_is_stepwise_binary32_not_fma(oracle, datagen):
    # On random inputs each Horner step must be the IEEE definition: the exact
    # product rounded to binary32, then the exact sum rounded to binary32.
    # Products and sums of two binary32 values are exact in double, so the
    # double operations below round only where binary32 rounds.  A fused
    # multiply-add (one rounding per step) differs on many of these inputs.
    x = datagen.fill(4096, 7, 0, 1, datagen.NORMAL)
    coef = np.float32([3.0, -1.25, 0.5])
    y = oracle.poly_map(x, coef)
    want = np.empty_like(x)
    fused_differs = 0
    for i, xi in enumerate(x.astype(np.float64)):
        t = np.float32(coef[2])
        tf = np.float32(coef[2])
        for k in (1, 0):
            p = np.float32(float(t) * xi)
            t = np.float32(float(p) + float(coef[k]))
            tf = np.float32(F(float(tf)) * F(xi) + F(float(coef[k])))
        want[i] = t
        fused_differs += int(tf != t)
    assert np.array_equal(y.view(np.uint32), want.view(np.uint32))
    assert fused_differs > 0  # the inputs do discriminate fused from unfused


def test_fmul_closed_form_dyadic(oracle):
    # x = a + i d, y = e + i f with dyadic steps and c = 0.25: all exact, so
    # z_i = x_i y_i + c x_i exactly; pins the operands (x*y + c*x, not c*y).
    i = np.arange(512)
    x = (-1.0 + i / 256.0).astype(np.float32)
    y = (0.5 + i / 128.0).astype(np.float32)
    z = oracle.fmul_map(x, y, 0.25)
    for xi, yi, zi in zip(x, y, z):
        assert frac32(zi) == frac32(xi) * frac32(yi) + F(1, 4) * frac32(xi)


def test_fmul_default_c_is_binary32_tenth(oracle, datagen):
    # c = 0.1 is the binary32 value 0x3DCCCCCD; z = round(round(xy)+round(cx)).
    c32 = np.float32(0.1)
    assert c32.view(np.uint32) == 0x3DCCCCCD
    x = datagen.fill(20000, 3, 1, 1, datagen.NORMAL)
    y = datagen.fill(20000, 3, 1, 2, datagen.U_02)
    z = oracle.fmul_map(x, y)
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    xy = (xd * yd).astype(np.float32)          # exact product, one rounding
    cx = (float(c32) * xd).astype(np.float32)  # exact product, one rounding
    want = (xy.astype(np.float64) + cx.astype(np.float64)).astype(np.float32)
    assert np.array_equal(z.view(np.uint32), want.view(np.uint32))
    # a fused x*y + cx (single rounding) disagrees on some of these inputs
    fused = np.array([np.float32(F(float(a)) * F(float(b)) + F(float(c)))
                      for a, b, c in zip(x[:2000], y[:2000], cx[:2000])])
    assert np.any(fused.view(np.uint32) != z[:2000].view(np.uint32))


def test_maps_empty(oracle):
    e = np.zeros(0, np.float32)
    assert oracle.poly_map(e, (1.0, 2.0)).size == 0
    assert oracle.fmul_map(e, e).size == 0
