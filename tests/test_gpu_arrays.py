"""GPU parity of the array-valued ReduceCL (sec. 3.1.3 item 3, Fig 3, sec.
3.2.2): sparkcl_reduce_arrays through the C ABI against the oracle's fixed
tree, bit for bit, over single- and multi-pass shapes, the float4 columns
(any 4-byte alignment) and the scalar ones (lengths not a multiple of 4),
both combiners, and the argument errors."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1505_01120_amd as sc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = sc.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.destroy()


def rdd(k: int, length: int, seed: int = 0, dist=None) -> np.ndarray:
    """k RDD elements of `length` floats; element e is stream (seed, e, tag 1)."""
    dist = datagen.NORMAL if dist is None else dist
    return np.stack([datagen.fill(length, seed, e, 1, dist) for e in range(k)]) \
        if k else np.zeros((0, length), np.float32)


def run(ctx, host: np.ndarray, combiner=sc.VADD, offset: int = 0, alias: bool = False):
    k, length = host.shape
    flat = torch.zeros(k * (length + offset) + 8, dtype=torch.float32, device="cuda")
    rows = []
    for e in range(k):
        r = flat[e * (length + offset) + offset:e * (length + offset) + offset + length]
        r.copy_(torch.from_numpy(host[e]))
        rows.append(r)
    out = rows[0] if alias else torch.full((length,), float("nan"), device="cuda")
    ctx.reduce_arrays(rows, out, combiner)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(ctx, host, combiner=sc.VADD, **kw):
    got = run(ctx, host, combiner, **kw)
    want = oracle.tree_reduce_arrays(host, combiner)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), \
        (host.shape, combiner, kw, int(np.sum(got.view(np.uint32) != want.view(np.uint32))))


# (k, len): one pass with full columns, ragged k around the 8-leaf groups,
# short arrays (several passes), long k, and float4-ragged lengths.
SHAPES = [(1, 1000), (2, 4096), (3, 4100), (7, 10_001), (8, 4096), (9, 4096),
          (17, 65_536), (64, 1 << 16), (300, 1024), (1000, 256), (5000, 64),
          (20_000, 16), (4097, 8)]


@pytest.mark.parametrize("k,length", SHAPES)
def test_vadd_matches_oracle(ctx, k, length):
    check(ctx, rdd(k, length, seed=k))


@pytest.mark.parametrize("k,length", [(5, 1001), (64, 4096), (3000, 32)])
def test_vmax_matches_oracle(ctx, k, length):
    check(ctx, rdd(k, length, seed=3), sc.VMAX)


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_unaligned_arrays(ctx, offset):
    # arrays (and their rows) 4, 8 or 12 bytes off a 16-byte boundary: float4
    # columns at 4-byte alignment; an odd length takes the scalar columns
    check(ctx, rdd(37, 4096, seed=offset), offset=offset)
    check(ctx, rdd(37, 4095, seed=offset), offset=offset)
    check(ctx, rdd(130, 1 << 20, seed=offset), offset=offset)


def test_ill_conditioned_tree_is_bit_exact(ctx):
    # large cancelling values make every combine round: the tree shape shows
    host = rdd(777, 2048, seed=9) * np.float32(1e3)
    host[::2] += np.float32(3e7)
    host[1::2] -= np.float32(3e7)
    check(ctx, host)


def test_out_may_alias_the_first_array(ctx):
    host = rdd(33, 4096, seed=4)
    got = run(ctx, host, alias=True)
    want = oracle.tree_reduce_arrays(host)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_repeat_uses_cached_plan_and_is_identical(ctx):
    host = rdd(100, 3000, seed=5)
    dev = [torch.from_numpy(r).cuda() for r in host]
    outs = []
    for _ in range(3):
        out = torch.empty(3000, device="cuda")
        ctx.reduce_arrays(dev, out)
        outs.append(out)
    torch.cuda.synchronize()
    want = oracle.tree_reduce_arrays(host)
    for o in outs:
        assert np.array_equal(o.cpu().numpy().view(np.uint32), want.view(np.uint32))


def test_full_size_64_arrays_of_2p22(ctx):
    # the 64 x 2^22 RDD as array-valued elements; every column bit-exact
    # against the oracle's tree
    k, length = 64, 1 << 22
    host = [datagen.fill(length, 0, e, 1, datagen.NORMAL) for e in range(k)]
    dev = torch.empty((k, length), dtype=torch.float32, device="cuda")
    for e in range(k):
        dev[e].copy_(torch.from_numpy(host[e]))
    out = torch.empty(length, device="cuda")
    for comb in (sc.VADD, sc.VMAX):
        ctx.reduce_arrays(list(dev), out, comb)
        torch.cuda.synchronize()
        want = oracle.tree_reduce_arrays(host, comb)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32)), comb


# Shapes that fill the GPU with float4 columns take the wide kernel (leaf
# pairs, 2 or 4 float4 columns per thread, chunks of 64 leaves): multi-pass
# with a ragged last chunk, an odd leaf at the end, and columns that end
# inside a block's span.  Grids of 512-thread blocks (2048 quads each) that
# give every CU two blocks (512 on 256 CUs) take its 512-thread form: the
# last two shapes,
# the second of them in two passes (its 65th leaf is a chunk of its own, and
# the pass over the two chunk rows takes the 256-thread form).  Columns are
# checked on samples against the oracle.
@pytest.mark.parametrize("k,length,comb", [(130, (1 << 20) + 4, sc.VADD),
                                           (77, (1 << 21) + 12, sc.VADD),
                                           (77, (1 << 21) + 12, sc.VMAX),
                                           (3, (1 << 21) + 4, sc.VADD),
                                           (200, 1 << 19, sc.VADD),
                                           (3, 4 * (2048 * 512 + 100), sc.VADD),
                                           (65, 4 * (2048 * 256 + 36), sc.VMAX)])
def test_wide_kernel_shapes(ctx, k, length, comb):
    dev = torch.empty((k, length), dtype=torch.float32, device="cuda")
    for e in range(k):
        dev[e].copy_(torch.from_numpy(datagen.fill(length, k, e, 1, datagen.NORMAL)))
    out = torch.full((length,), float("nan"), device="cuda")
    ctx.reduce_arrays(list(dev), out, comb)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for lo in (0, 4096 * 3 + 8, length // 2 - 100, length - 5000):
        want = oracle.tree_reduce_arrays(dev[:, lo:lo + 5000].cpu().numpy(), comb)
        assert np.array_equal(got[lo:lo + 5000].view(np.uint32), want.view(np.uint32)), (k, lo)


def test_errors(ctx):
    x = torch.zeros(64, device="cuda")
    out = torch.zeros(64, device="cuda")
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_arrays([], out)
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_arrays([x, x], out, combiner=9)
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_arrays([x, 0], out)
    assert e.value.code == sc.EINVAL
    with pytest.raises(sc.SparkclError) as e:
        ctx.reduce_arrays([x, x.data_ptr() + 2], out)
    assert e.value.code == sc.EINVAL
    # nothing to do for empty arrays
    ctx.reduce_arrays([x[:0], x[:0]], out[:0])


# ---- rows of one buffer (sparkcl_reduce_rows) ---------------------------------

@pytest.mark.parametrize("k,length,pad", [(1, 100, 0), (9, 4096, 0), (64, 65_536, 1024),
                                          (150, (1 << 20) + 8, 4),
                                          (300, 1000, 3), (65_536, 64, 0),
                                          (1 << 20, 16, 0), (5000, 12, 4)])
def test_rows_match_oracle(ctx, k, length, pad):
    host = rdd(k, length, seed=k + pad) if k * length <= (1 << 22) else \
        datagen.fill(k * length, 7, 0, 1, datagen.NORMAL).reshape(k, length)
    buf = torch.zeros(k * (length + pad), dtype=torch.float32, device="cuda")
    rows = buf.view(k, length + pad)[:, :length]
    rows.copy_(torch.from_numpy(host))
    out = torch.full((length,), float("nan"), device="cuda")
    for comb in (sc.VADD, sc.VMAX):
        ctx.reduce_rows(rows, out, comb)
        torch.cuda.synchronize()
        want = oracle.tree_reduce_arrays(host, comb)
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (k, length, pad, comb)


def oracle_by_column_blocks(host, comb, blocks=16):
    """The oracle's tree over the rows of `host`, run on blocks of columns in
    parallel host threads (each column's tree is independent of the others)."""
    from concurrent.futures import ThreadPoolExecutor
    n = host.shape[1]
    step = -(-n // blocks)
    with ThreadPoolExecutor(blocks) as ex:
        parts = list(ex.map(lambda lo: oracle.tree_reduce_rows(host[:, lo:lo + step], comb),
                            range(0, n, step)))
    return np.concatenate(parts)


def test_rows_full_size_65536_of_4096(ctx):
    # The 1 GiB RDD as 65536 rows of 4096 floats (the benchmark's second
    # array shape, three passes of the 8-leaf kernel); both combiners, every
    # column bit-exact against the oracle's tree over all 65536 rows
    k, length = 65_536, 4096
    host = datagen.fill(k * length, 11, 0, 1, datagen.NORMAL).reshape(k, length)
    rows = torch.from_numpy(host).cuda()
    out = torch.full((length,), float("nan"), device="cuda")
    for comb in (sc.VADD, sc.VMAX):
        ctx.reduce_rows(rows, out, comb)
        torch.cuda.synchronize()
        want = oracle_by_column_blocks(host, comb)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32)), comb


def test_rows_errors(ctx):
    buf = torch.zeros(64, device="cuda")
    out = torch.zeros(16, device="cuda")
    L = sc.load()
    rc = L.sparkcl_reduce_rows(ctx._h, sc.VADD, buf.data_ptr(), 8, 4, 16, out.data_ptr(), None)
    assert rc == sc.EINVAL                                    # stride below the length
    rc = L.sparkcl_reduce_rows(ctx._h, sc.VADD, buf.data_ptr() + 2, 16, 4, 16, out.data_ptr(), None)
    assert rc == sc.EINVAL                                    # misaligned rows
    rc = L.sparkcl_reduce_rows(ctx._h, sc.VADD, None, 16, 4, 16, out.data_ptr(), None)
    assert rc == sc.EINVAL
