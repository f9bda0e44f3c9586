"""Pin of the oracle's map-chain composition: on dyadic inputs where every
binary32 step is exact, the chain equals the composed polynomial evaluated
in FP64 (a closed form), and stages apply in the listed order."""
import numpy as np


def test_chain_closed_form(oracle):
    x = (np.arange(-64, 64) / 4).astype(np.float32)          # k/4, exact
    y = (np.arange(128) % 7 / 2).astype(np.float32)           # j/2, exact
    # FMUL with c = 0.25, then 1 + 2v, then v^2 / 4: all exact on this grid
    got = oracle.chain_map(x, y, 2, c=np.float32(0.25), stages=[(1.0, 2.0), (0.0, 0.0, 0.25)])
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    v = xd * yd + 0.25 * xd
    v = 1.0 + 2.0 * v
    v = 0.25 * v * v
    assert np.array_equal(got.astype(np.float64), v)
    # order matters: the two stages swapped give a different closed form
    swapped = oracle.chain_map(x, y, 2, c=np.float32(0.25), stages=[(0.0, 0.0, 0.25), (1.0, 2.0)])
    w = xd * yd + 0.25 * xd
    w = 1.0 + 2.0 * (0.25 * w * w)
    assert np.array_equal(swapped.astype(np.float64), w)
    assert not np.array_equal(got, swapped)


def test_empty_chain_is_the_task_map(oracle):
    x = np.linspace(-1, 1, 1001, dtype=np.float32)
    coef = (3.0, -1.25, 0.5)
    assert np.array_equal(oracle.chain_map(x, None, 1, coef), oracle.poly_map(x, coef))
