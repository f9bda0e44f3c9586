"""Pins of the oracle's array-valued ReduceCL (O9; sec. 3.1.3 item 3, Fig 3,
sec. 3.2.2): RDD elements that are float arrays, folded with a two-input
combiner kernel along a fixed pairwise tree."""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
U = 2.0 ** -24


def level_pairing(rows):
    """The same tree described level by level: combine neighbours (0,1),
    (2,3), ... with numpy's float32 add, carry an odd last element up
    unchanged, repeat until one row is left."""
    rows = [np.asarray(r, dtype=np.float32) for r in rows]
    while len(rows) > 1:
        nxt = [rows[i] + rows[i + 1] for i in range(0, len(rows) - 1, 2)]
        if len(rows) % 2:
            nxt.append(rows[-1])
        rows = nxt
    return rows[0]


def test_tree_equals_level_pairing(oracle):
    rng = np.random.default_rng(11)
    for k in list(range(1, 70)) + [127, 128, 129, 255, 256, 257, 1000]:
        a = (rng.standard_normal((k, 24)) *
             np.exp(rng.uniform(-20, 20, (k, 1)))).astype(np.float32)
        got = oracle.tree_reduce_arrays(a)
        want = level_pairing(list(a))
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), k


def test_worked_examples(oracle):
    with open(os.path.join(HERE, "golden", "tree_reduce_examples.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        rows = [np.float32([v]) for v in c["elements"]]
        got = float(oracle.tree_reduce_arrays(rows)[0])
        assert got == c["expect"], c["derivation"]
        for name, v in c["not"].items():
            assert got != v, name


def test_integer_inputs_are_exact(oracle):
    # every partial sum stays below 2^24 in magnitude, so any order is exact
    rng = np.random.default_rng(5)
    for k in (1, 2, 3, 17, 64, 1000):
        a = rng.integers(-1000, 1000, size=(k, 40))
        got = oracle.tree_reduce_arrays(a.astype(np.float32))
        assert np.array_equal(got, a.sum(axis=0).astype(np.float32)), k


def test_vmax_is_the_columnwise_max(oracle):
    rng = np.random.default_rng(6)
    for k in (1, 2, 5, 33, 300):
        a = rng.standard_normal((k, 50)).astype(np.float32)
        got = oracle.tree_reduce_arrays(a, oracle.VMAX)
        assert np.array_equal(got, a.max(axis=0)), k


def test_pairwise_error_bound(oracle):
    # Pairwise summation: |fl - exact| <= gamma_h * sum|a|, h = ceil(log2 K)
    # (Higham, Accuracy and Stability of Numerical Algorithms, sec. 4.2).  A
    # bound, not a shape test: the worked examples and the level pairing pin
    # the shape.
    rng = np.random.default_rng(7)
    for k in (2, 3, 100, 1024, 3000):
        a = (rng.standard_normal((k, 64)) * 1e3).astype(np.float32)
        a[:, ::2] += 1e6                      # large cancelling offsets
        a[1::2, ::2] -= 2e6
        got = oracle.tree_reduce_arrays(a)
        h = math.ceil(math.log2(k))
        gamma = h * U / (1 - h * U)
        for i in range(a.shape[1]):
            col = a[:, i].astype(np.float64)
            exact = math.fsum(col)
            assert abs(float(got[i]) - exact) <= gamma * np.abs(col).sum(), (k, i)


def test_single_element_is_copied_and_errors(oracle):
    a = np.float32([[1.5, -0.0, np.inf]])
    got = oracle.tree_reduce_arrays(a)
    assert np.array_equal(got.view(np.uint32), a[0].view(np.uint32))
    with pytest.raises(ValueError):
        oracle.tree_reduce_arrays([])
    with pytest.raises(ValueError):
        oracle.tree_reduce_arrays(a, 9)
    assert oracle.tree_reduce_arrays(np.zeros((3, 0), np.float32)).size == 0


def test_rows_entry_is_the_same_fold(oracle):
    # tree_reduce_rows only builds the row pointers differently: on strided
    # column windows of a larger array it returns the per-array fold's bits
    rng = np.random.default_rng(3)
    big = rng.standard_normal((131, 70)).astype(np.float32)
    for comb in (oracle.VADD, oracle.VMAX):
        for lo, hi in ((0, 70), (5, 41), (69, 70)):
            want = oracle.tree_reduce_arrays([r[lo:hi] for r in big], comb)
            got = oracle.tree_reduce_rows(big[:, lo:hi], comb)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (comb, lo, hi)
    with pytest.raises(ValueError):
        oracle.tree_reduce_rows(big.astype(np.float64))
    with pytest.raises(ValueError):
        oracle.tree_reduce_rows(big[:, ::2])
    with pytest.raises(ValueError):
        oracle.tree_reduce_rows(big[:0])
