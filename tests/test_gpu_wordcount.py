"""GPU parity of WordCount (sec. 3.2.3): sparkcl_wordcount through the C
ABI against the oracle, exactly: the same distinct keys with the same counts
(the GPU's output order is free, so both sides are compared sorted by key)
and the same number of words."""
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


def gpu_count(ctx, text: np.ndarray, offset: int = 0, capacity=None):
    buf = torch.zeros(text.size + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + text.size]
    view.copy_(torch.from_numpy(text))
    cap = capacity if capacity is not None else text.size // 2 + 1
    keys, counts, nd, nw = ctx.wordcount(view, cap)
    k = keys[:nd].cpu().numpy().view(np.uint64)
    c = counts[:nd].cpu().numpy().view(np.uint64)
    order = np.argsort(k)
    return k[order], c[order], nw


def check(ctx, text, offset=0):
    text = np.frombuffer(text, dtype=np.uint8) if isinstance(text, bytes) else text
    gk, gc, gn = gpu_count(ctx, text, offset)
    ok, oc, on = oracle.wordcount(text)
    assert gn == on, (gn, on)
    assert np.array_equal(gk, ok) and np.array_equal(gc, oc)


EDGE = [b"", b"a", b" ", b"  a  ", b"a b\tc\nd\re\x0bf\x0cg", b"\x00\x01 \x7f\xff",
        b"x" * 10_000, b" \t\n\r\x0b\x0c" * 100]


@pytest.mark.parametrize("i", range(len(EDGE)))
def test_edge_texts(ctx, i):
    check(ctx, EDGE[i])


@pytest.mark.parametrize("n", [4095, 4096, 4097, 4351, 4352, 4353, 8192 + 7])
def test_words_across_chunk_and_lookahead_edges(ctx, n):
    # words of every length 1..600 laid end to end, cut at n bytes
    parts, rng = [], np.random.default_rng(n)
    while sum(map(len, parts)) < n:
        parts.append(b"q" * int(rng.integers(1, 600)) + b" ")
    check(ctx, b"".join(parts)[:n])


@pytest.mark.parametrize("offset", [0, 1, 7, 15])
def test_random_bytes_any_alignment(ctx, offset):
    rng = np.random.default_rng(offset)
    check(ctx, rng.integers(0, 256, (1 << 20) + 13, dtype=np.uint8), offset)


@pytest.mark.parametrize("vocab,nbytes", [(10, 1 << 20), (20_000, 8 << 20), (1_000_000, 16 << 20)])
def test_zipf_corpus(ctx, vocab, nbytes):
    check(ctx, datagen.corpus(nbytes, vocab=vocab, seed=vocab))


def test_capacity_overflow(ctx):
    text = datagen.corpus(1 << 20, vocab=20_000)
    ok, _, _ = oracle.wordcount(text)
    cap = len(ok) - 1
    buf = torch.from_numpy(text).cuda()
    with pytest.raises(sc.SparkclError) as e:
        ctx.wordcount(buf, cap)
    assert e.value.code == sc.ETOOBIG
    # exactly enough room succeeds
    keys, counts, nd, nw = ctx.wordcount(buf, len(ok))
    assert nd == len(ok)


def test_full_size_1gib(ctx):
    # The benchmark's 1 GiB text: a 64 MiB Zipf corpus (vocabulary 10^5,
    # ending in a newline, so no word spans two copies) repeated 16 times.
    # Same keys as the oracle on the base, every count and the word total
    # 16 times the base's.
    base_n, rep = 64 << 20, 16
    base = datagen.corpus(base_n - 1, vocab=100_000)
    base = np.concatenate([base, np.frombuffer(b"\n", dtype=np.uint8)])
    text = torch.from_numpy(base).cuda().repeat(rep)
    ok, oc, on = oracle.wordcount(base)
    keys, counts, nd, nw = ctx.wordcount(text, 1 << 20)  # the benchmark's capacity
    k = keys[:nd].cpu().numpy().view(np.uint64)
    c = counts[:nd].cpu().numpy().view(np.uint64)
    order = np.argsort(k)
    assert nw == rep * on, (nw, rep * on)
    assert np.array_equal(k[order], ok)
    assert np.array_equal(c[order], oc * np.uint64(rep))


# An 8-byte word whose FNV-1a 64 key is 0, the GPU table's empty-slot value
# (the oracle's pins derive the key from the definition).  The GPU counts it
# in a counter of its own and emits it at compaction; these texts put it at
# span (16-byte), chunk (4096) and look-ahead (256) edges, at the text's end,
# repeated, among a skewed vocabulary and at unaligned text addresses.
ZERO_KEY_WORD = bytes.fromhex("d56bb95342870836")


def filler(n: int, seed: int) -> bytearray:
    rng = np.random.default_rng(seed)
    t = rng.choice(np.frombuffer(b"abcdefgh  \n", dtype=np.uint8), n)
    return bytearray(t.tobytes())


def put_zero_word(t: bytearray, pos: int) -> None:
    if pos > 0:
        t[pos - 1] = 0x20
    t[pos:pos + 8] = ZERO_KEY_WORD
    if pos + 8 < len(t):
        t[pos + 8] = 0x0A


@pytest.mark.parametrize("pos", [0, 5, 8, 12, 15, 16, 4088, 4090, 4095, 4096, 4096 + 248,
                                 4096 + 250, 8191, 8192 + 4096 - 3])
def test_zero_key_word_positions(ctx, pos):
    t = filler(pos + 300, pos)
    put_zero_word(t, pos)
    check(ctx, bytes(t))


@pytest.mark.parametrize("offset", [0, 1, 7])
def test_zero_key_word_at_text_end_and_alone(ctx, offset):
    check(ctx, ZERO_KEY_WORD, offset)
    t = filler(5000, 1)
    t[-9] = 0x20
    t[-8:] = ZERO_KEY_WORD
    check(ctx, bytes(t), offset)


def test_zero_key_word_repeated_in_corpus(ctx):
    # many copies, each block of the grid sees some; the key-0 count is the
    # sum over blocks
    base = bytearray(datagen.corpus(4 << 20, vocab=20_000, seed=5).tobytes())
    rng = np.random.default_rng(9)
    for pos in sorted(rng.choice(len(base) - 16, 3000, replace=False)):
        put_zero_word(base, int(pos) + 1)
    check(ctx, bytes(base))
    check(ctx, (ZERO_KEY_WORD + b" ") * 10_000)


def _one_partition_words(count: int, length: int = 8, seed: int = 5) -> np.ndarray:
    """`count` distinct lowercase words of `length` letters whose 64-bit FNV-1a
    keys all have a top byte of 0 (the oracle's hash, computed here with
    numpy's wrapping uint64 arithmetic and checked against the oracle), as
    rows of a uint8 array."""
    rng = np.random.default_rng(seed)
    out = []
    with np.errstate(over="ignore"):
        while sum(len(o) for o in out) < count:
            w = rng.integers(ord("a"), ord("z") + 1, (1 << 20, length), dtype=np.uint8)
            h = np.full(w.shape[0], 14695981039346656037, dtype=np.uint64)
            for j in range(length):
                h = (h ^ w[:, j].astype(np.uint64)) * np.uint64(1099511628211)
            out.append(w[(h >> np.uint64(56)) == 0])
    w = np.unique(np.concatenate(out), axis=0)[:count]
    ok, _, _ = oracle.wordcount(np.concatenate([np.append(r, 32) for r in w[:4]]).astype(np.uint8))
    assert np.all((ok >> np.uint64(56)) == 0)
    return w


def test_spill_regions_of_one_partition_overflow(ctx):
    # 1500 distinct words whose keys share their top byte, so every word that
    # misses a block's LDS table (1024 slots; each block scans 16 chunks)
    # spills into the same partition's region, which overflows: the excess
    # goes to the table directly, the rest through the merge.
    w = _one_partition_words(1500)
    rng = np.random.default_rng(11)
    line = np.concatenate([np.append(w[i], 32) for i in rng.integers(0, len(w), 1 << 16)])
    reps = (64 << 20) // line.size + 1
    text = np.tile(line.astype(np.uint8), reps)[:64 << 20]
    gk, gc, gn = gpu_count(ctx, text, capacity=1 << 14)
    ok, oc, on = oracle.wordcount(text)
    assert gn == on, (gn, on)
    assert np.array_equal(gk, ok) and np.array_equal(gc, oc)


# ---- the first occurrence of each key (sparkcl_wordcount_locate) -------------

def check_locate(ctx, text, offset=0, extra_keys=()):
    """Count on the GPU, then locate every key it returned (and `extra_keys`,
    which the text need not hold): each offset equal to the oracle's first
    occurrence, UINT64_MAX for absent keys."""
    text = np.frombuffer(text, dtype=np.uint8) if isinstance(text, bytes) else text
    buf = torch.zeros(text.size + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + text.size]
    view.copy_(torch.from_numpy(text))
    keys, counts, nd, nw = ctx.wordcount(view, text.size // 2 + 1)
    q = np.concatenate([keys[:nd].cpu().numpy().view(np.uint64),
                        np.array(extra_keys, dtype=np.uint64)])
    qd = torch.from_numpy(q.view(np.int64).copy()).cuda()
    off = ctx.wordcount_locate(view, qd, q.size).cpu().numpy()[:q.size].view(np.uint64)
    want = oracle.wordcount_first(text, q)
    assert np.array_equal(off, want), np.nonzero(off != want)[0][:10]
    return q, off


@pytest.mark.parametrize("i", range(len(EDGE)))
def test_locate_edge_texts(ctx, i):
    check_locate(ctx, EDGE[i])


@pytest.mark.parametrize("n", [4095, 4097, 4353, 8192 + 7])
def test_locate_across_chunk_and_lookahead_edges(ctx, n):
    parts, rng = [], np.random.default_rng(n)
    while sum(map(len, parts)) < n:
        parts.append(b"q" * int(rng.integers(1, 600)) + b" ")
    check_locate(ctx, b"".join(parts)[:n])


@pytest.mark.parametrize("offset", [0, 3])
def test_locate_random_bytes_and_absent_keys(ctx, offset):
    rng = np.random.default_rng(offset + 40)
    text = rng.integers(0, 256, (1 << 20) + 13, dtype=np.uint8)
    absent = [oracle.fnv1a64(b"\x20"), 1, 2**64 - 1]   # no word hashes to these here
    q, off = check_locate(ctx, text, offset, absent)
    assert off[-2:].tolist() == [2**64 - 1, 2**64 - 1]


@pytest.mark.parametrize("vocab,nbytes", [(10, 1 << 20), (20_000, 8 << 20), (1_000_000, 16 << 20)])
def test_locate_zipf_corpus(ctx, vocab, nbytes):
    check_locate(ctx, datagen.corpus(nbytes, vocab=vocab, seed=vocab + 1))


@pytest.mark.parametrize("pos", [0, 15, 4095, 4096 + 250])
def test_locate_zero_key_word(ctx, pos):
    t = filler(pos + 300, pos + 1)
    put_zero_word(t, pos)
    put_zero_word(t, pos + 100)   # a second copy: the first one counts
    q, off = check_locate(ctx, bytes(t))
    assert off[q.tolist().index(0)] == pos


def test_locate_errors_and_empty(ctx):
    text = torch.from_numpy(np.frombuffer(b"ab cd ab", dtype=np.uint8).copy()).cuda()
    k = oracle.fnv1a64(b"ab")
    dup = torch.from_numpy(np.array([k, k], dtype=np.uint64).view(np.int64)).cuda()
    with pytest.raises(sc.SparkclError) as e:
        ctx.wordcount_locate(text, dup, 2)
    assert e.value.code == sc.EINVAL
    zero = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(sc.SparkclError) as e:
        ctx.wordcount_locate(text, zero, 2)       # the key 0 twice
    assert e.value.code == sc.EINVAL
    one = torch.from_numpy(np.array([k], dtype=np.uint64).view(np.int64)).cuda()
    assert ctx.wordcount_locate(text, one, 1).cpu().tolist() == [0]
    empty = torch.zeros(0, dtype=torch.uint8, device="cuda")
    assert ctx.wordcount_locate(empty, one, 1).cpu().numpy().view(np.uint64).tolist() == \
        [2**64 - 1]
    ctx.wordcount_locate(text, one, 0)            # no keys: nothing to do


def test_locate_full_size_1gib(ctx):
    # The benchmark's 1 GiB text (the 64 MiB base repeated 16 times): every
    # key's first word lies in the first copy, at the oracle's offset on the
    # base.
    base_n, rep = 64 << 20, 16
    base = datagen.corpus(base_n - 1, vocab=100_000)
    base = np.concatenate([base, np.frombuffer(b"\n", dtype=np.uint8)])
    text = torch.from_numpy(base).cuda().repeat(rep)
    keys, counts, nd, nw = ctx.wordcount(text, 1 << 20)
    off = ctx.wordcount_locate(text, keys, nd).cpu().numpy()[:nd].view(np.uint64)
    k = keys[:nd].cpu().numpy().view(np.uint64)
    assert np.array_equal(off, oracle.wordcount_first(base, k))
