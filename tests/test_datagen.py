"""The seeded input generator: determinism, exactness of the uniform grids and
the shape of the workload recipes."""
import math

import numpy as np


def test_deterministic_and_thread_independent(datagen, monkeypatch):
    a = datagen.fill(1 << 18, 0, 5, 1, datagen.NORMAL)
    monkeypatch.setattr(datagen, "_threads", lambda: 1)
    b = datagen.fill(1 << 18, 0, 5, 1, datagen.NORMAL)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    # a prefix of a longer stream equals the shorter stream
    c = datagen.fill(1000, 0, 5, 1, datagen.NORMAL)
    assert np.array_equal(a[:1000].view(np.uint32), c.view(np.uint32))


def test_streams_differ(datagen):
    x = datagen.fill(64, 0, 0, 1, datagen.WORDS)
    assert not np.array_equal(x, datagen.fill(64, 0, 1, 1, datagen.WORDS))
    assert not np.array_equal(x, datagen.fill(64, 0, 0, 2, datagen.WORDS))
    assert not np.array_equal(x, datagen.fill(64, 1, 0, 1, datagen.WORDS))


def test_uniform_grids_exact(datagen):
    x = datagen.fill(1 << 16, 0, 0, 1, datagen.U_PM1)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert np.all((x.astype(np.float64) * 2 ** 23) % 1 == 0)
    y = datagen.fill(1 << 16, 0, 0, 2, datagen.U_02)
    assert y.min() >= 0.0 and y.max() < 2.0
    assert np.all((y.astype(np.float64) * 2 ** 23) % 1 == 0)


def test_normal_moments(datagen):
    z = datagen.fill(1 << 20, 0, 0, 1, datagen.NORMAL).astype(np.float64)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 0.01
    assert np.all(np.isfinite(z))


def test_workload_recipes(datagen):
    sizes, kids = datagen.uneven_sizes()
    assert sizes.size == 4096 and sizes.min() >= 1024 and sizes.max() <= 8388608
    assert set(np.unique(kids)) == {1, 2, 3}
    med = np.median(sizes)
    assert 50000 < med < 85000
    tr = datagen.serving_trace(20000, pool=1 << 24)
    rate = tr.t_arrive.size / tr.t_arrive[-1]
    assert 19000 < rate < 21000
    assert tr.sizes.max() <= 4194304 and tr.sizes.min() >= 1024
    assert np.all(tr.offsets + tr.sizes <= (1 << 24)) and np.all(tr.offsets % 64 == 0)
    parts = datagen.fmul_rdd(parts=2, n=1000)
    assert parts[0].x.dtype == np.float32 and parts[1].y.size == 1000
    assert not np.array_equal(parts[0].x, parts[1].x)
