"""The bench's read-ceiling kernel (libsparkcl_probe.so): it reads every
element of both arrays exactly once, so the per-block sums add up to the sum
of x + y; bad shapes are refused and launch nothing."""
import ctypes
import os

import numpy as np
import pytest
import torch

import paper_1505_01120_amd as sc
from paper_1505_01120_amd import build as libbuild

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def probe():
    lib = ctypes.CDLL(libbuild.PROBE_LIB)
    fn = lib.sparkcl_probe_read2
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                   ctypes.c_void_p, ctypes.c_void_p]
    return fn


@pytest.mark.parametrize("grid,passes", [(1, 1), (256, 3), (1024, 2)])
def test_every_element_read_once(probe, grid, passes):
    n = 4096 * grid * passes
    g = torch.Generator().manual_seed(grid)
    # small integers: every partial sum is exact in binary32
    x = torch.randint(-8, 9, (n,), generator=g).float().cuda()
    y = torch.randint(-8, 9, (n,), generator=g).float().cuda()
    sink = torch.full((grid,), float("nan"), device="cuda")
    assert probe(x.data_ptr(), y.data_ptr(), n, grid, sink.data_ptr(),
                 torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    want = float(x.double().sum() + y.double().sum())
    assert not torch.isnan(sink).any()
    assert float(sink.double().sum()) == want


def test_bad_shapes_launch_nothing(probe):
    x = torch.zeros(8192, device="cuda")
    sink = torch.full((4,), 7.0, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert probe(x.data_ptr(), x.data_ptr(), 4096 * 3, 2, sink.data_ptr(), s) == sc.EINVAL
    assert probe(x.data_ptr() + 4, x.data_ptr(), 4096, 1, sink.data_ptr(), s) == sc.EINVAL
    torch.cuda.synchronize()
    assert torch.equal(sink, torch.full((4,), 7.0, device="cuda"))
