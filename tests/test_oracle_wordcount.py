"""Pins of the oracle's WordCount (O10; sec. 3.2.3): the FNV-1a 64 key
against its published test vectors, and tokenisation and counting against
Python's own whitespace split and collections.Counter."""
from collections import Counter

import numpy as np


def by_key(oracle, words):
    c = Counter(words)
    pairs = sorted((oracle.fnv1a64(w), n) for w, n in c.items())
    return [k for k, _ in pairs], [n for _, n in pairs]


def test_fnv1a64_published_vectors(oracle):
    # Fowler/Noll/Vo FNV-1a, 64-bit: empty string, "a", "foobar"
    assert oracle.fnv1a64(b"") == 0xCBF29CE484222325
    assert oracle.fnv1a64(b"a") == 0xAF63DC4C8601EC8C
    assert oracle.fnv1a64(b"foobar") == 0x85944171F73967E8


def check(oracle, text: bytes):
    keys, counts, nw = oracle.wordcount(text)
    words = text.split()      # Python splits bytes on the same six whitespace bytes
    k, n = by_key(oracle, words)
    assert nw == len(words)
    assert keys.tolist() == k and counts.tolist() == n
    assert len(set(k)) == len(set(words))   # no key collisions in these inputs


def test_edge_texts(oracle):
    for t in [b"", b"a", b" ", b"  a  ", b"a b\tc\nd\re\x0bf\x0cg", b"\x00\x01 \x7f\xff",
              b"x" * 5000, b"ab ab  ab\n\nab", b" \t\n\r\x0b\x0c" * 10]:
        check(oracle, t)


def test_random_bytes(oracle):
    rng = np.random.default_rng(3)
    check(oracle, rng.integers(0, 256, 1 << 16, dtype=np.uint8).tobytes())
    # mostly spaces: many one- and two-byte words
    t = rng.choice(np.frombuffer(b"  \n\tab", dtype=np.uint8), 1 << 16)
    check(oracle, t.tobytes())


def test_synthetic_corpus(oracle, datagen):
    text = datagen.corpus(1 << 20, vocab=20_000)
    check(oracle, text.tobytes())


# An 8-byte word, with no whitespace byte, whose 64-bit FNV-1a key is 0 (the
# value the GPU's counting table uses for an empty slot, so the GPU counts it
# apart).  Its key is derived here from the FNV-1a definition by hand: 64-bit
# offset basis, then for each byte xor it in and multiply by the prime mod 2^64.
ZERO_KEY_WORD = bytes.fromhex("d56bb95342870836")


def test_zero_key_word(oracle):
    h = 0xCBF29CE484222325
    for b in ZERO_KEY_WORD:
        h = ((h ^ b) * 0x100000001B3) % (1 << 64)
    assert h == 0
    assert not any(b in b" \t\n\x0b\x0c\r" for b in ZERO_KEY_WORD)
    assert oracle.fnv1a64(ZERO_KEY_WORD) == 0
    text = b"ab " + ZERO_KEY_WORD + b"\n" + ZERO_KEY_WORD + b" cd ab " + ZERO_KEY_WORD
    check(oracle, text)
    keys, counts, nw = oracle.wordcount(text)
    assert keys[0] == 0 and counts[0] == 3 and nw == 6


# ---- the first occurrence of each key ----------------------------------------

def first_by_regex(oracle, text: bytes) -> dict:
    """key -> byte offset of the first word with that key, from Python's
    regular-expression tokenisation (runs of bytes outside the six whitespace
    bytes) and a plain dictionary that keeps each word's first start."""
    import re
    first = {}
    for m in re.finditer(rb"[^ \t\n\x0b\x0c\r]+", text):
        first.setdefault(m.group(0), m.start())
    return {oracle.fnv1a64(w): off for w, off in first.items()}


def check_first(oracle, text: bytes):
    want = first_by_regex(oracle, text)
    keys = np.array(sorted(want), dtype=np.uint64)
    got = oracle.wordcount_first(text, keys)
    assert got.tolist() == [want[int(k)] for k in keys]
    # every word's offset names a word with that key
    for k, off in zip(keys.tolist(), got.tolist()):
        end = off
        while end < len(text) and text[end] not in b" \t\n\x0b\x0c\r":
            end += 1
        assert oracle.fnv1a64(text[off:end]) == k
        assert off == 0 or text[off - 1] in b" \t\n\x0b\x0c\r"


def test_first_occurrence_edge_texts(oracle):
    for t in [b"a", b"  a  ", b"a b\tc\nd\re\x0bf\x0cg", b"ab ab  ab\n\nab", b"b a b a c",
              b"x" * 5000, b"\x00\x01 \x7f\xff \x00\x01"]:
        check_first(oracle, t)
    text = b"ab " + ZERO_KEY_WORD + b"\n" + ZERO_KEY_WORD + b" cd"
    got = oracle.wordcount_first(text, np.array([0], dtype=np.uint64))
    assert got.tolist() == [3]


def test_first_occurrence_absent_and_empty(oracle):
    absent = np.array([oracle.fnv1a64(b"zz"), 12345], dtype=np.uint64)
    assert oracle.wordcount_first(b"a b c", absent).tolist() == [2**64 - 1] * 2
    assert oracle.wordcount_first(b"", absent).tolist() == [2**64 - 1] * 2
    assert oracle.wordcount_first(b"a", np.array([], dtype=np.uint64)).size == 0


def test_first_occurrence_corpus(oracle, datagen):
    text = datagen.corpus(1 << 18, vocab=5_000).tobytes()
    check_first(oracle, text)
