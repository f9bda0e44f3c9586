"""The bench's probe kernels (libsparkcl_probe.so).  The read-ceiling kernel
reads every element of both arrays exactly once, so the per-block sums add up
to the sum of x + y; bad shapes are refused and launch nothing.  The VALU
ceiling's Philox loop draws the same pairs as a Monte-Carlo partition, so its
hit counts add up to the oracle's count for that partition."""
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


@pytest.mark.parametrize("mix,grid,iters,seed,pid", [(0, 4, 8, 0, 0), (0, 3, 5, 0x1234567890ABCDEF, 77),
                                                    (1, 2, 6, 42, 3)])
def test_valu_probe_draws_the_partition_pairs(oracle, mix, grid, iters, seed, pid):
    fn = ctypes.CDLL(libbuild.PROBE_LIB).sparkcl_probe_valu
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    sink = torch.full((grid * 256,), -1, dtype=torch.int32, device="cuda")
    clk = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert fn(mix, grid, iters, seed, pid, sink.data_ptr(), clk.data_ptr(),
              torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    pairs = grid * 256 * iters * (2 if mix == 1 else 1)
    want = oracle.mc_count(seed, pid, 2 * pairs)
    assert int(sink.long().sum()) == want
    c = clk.cpu().tolist()
    assert c[2] > c[0] and c[3] > c[1]          # block 0's clock marks advanced


def test_clock_rates():
    fn = ctypes.CDLL(libbuild.PROBE_LIB).sparkcl_probe_clock_rates
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    assert fn(0, ctypes.byref(a), ctypes.byref(b)) == 0
    assert 1_000_000 < a.value < 5_000_000      # peak shader clock in kHz
    assert 0 < b.value < a.value                # the wall clock is slower
