"""CPU tests of the library's host side: the C ABI surface (every declared
symbol exported, struct layouts as the header defines them, clean failure
without a GPU) and the pure host logic behind it: the arena sub-allocator,
serving admission control and the tuning table with its JSON cache."""
import ctypes
import hashlib
import json
import os
import re
import subprocess

import pytest

import paper_1505_01120_amd as sc
from paper_1505_01120_amd import build as libbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparkcl.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    return sc.load()


@pytest.fixture(scope="module")
def host():
    if not os.path.exists(libbuild.HOST_LIB):
        libbuild.build()
    H = ctypes.CDLL(libbuild.HOST_LIB)
    U64, U32, P = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    for name, args, res in [
        ("hl_arena_new", [U64], P), ("hl_arena_free", [P], None),
        ("hl_arena_alloc", [P, U64], U64), ("hl_arena_release", [P, U64], ctypes.c_int),
        ("hl_arena_in_use", [P], U64), ("hl_arena_peak", [P], U64),
        ("hl_arena_largest_free", [P], U64), ("hl_arena_free_blocks", [P], U64),
        ("hl_arena_live_blocks", [P], U64), ("hl_arena_size", [P], U64),
        ("hl_adm_new", [U64, U32, U64], P), ("hl_adm_free", [P], None),
        ("hl_adm_fits", [P, U64, U32], ctypes.c_int),
        ("hl_adm_push", [P, U64, U64, U32, U64], None),
        ("hl_adm_head_block", [P], ctypes.c_int),
        ("hl_adm_admit", [P, ctypes.POINTER(U64), ctypes.POINTER(U32), ctypes.POINTER(U64)],
         ctypes.c_int),
        ("hl_adm_unadmit", [P, U64], ctypes.c_int), ("hl_adm_complete", [P, U64], ctypes.c_int),
        ("hl_adm_in_use", [P], U64), ("hl_adm_peak", [P], U64), ("hl_adm_pending", [P], U64),
        ("hl_adm_in_flight", [P], U64), ("hl_adm_tiles", [P], U64),
        ("hl_adm_push_staged", [P, U64, U64, U32, U64], None),
        ("hl_adm_take_slot", [P, U64, ctypes.POINTER(U64), ctypes.POINTER(U32)], ctypes.c_int),
        ("hl_adm_unadmit_staged", [P, U64], ctypes.c_int),
        ("hl_adm_complete_staged", [P, U64], ctypes.c_int),
        ("hl_tuning_defaults", [ctypes.POINTER(sc.Tuning)], None),
        ("hl_tuning_validate", [ctypes.POINTER(sc.Tuning)], ctypes.c_int),
        ("hl_tile_for", [ctypes.POINTER(sc.Tuning), ctypes.c_int, U32, U64], U32),
        ("hl_size_bucket", [U64], U32),
        ("hl_tuning_save", [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(sc.Tuning)],
         ctypes.c_int),
        ("hl_tuning_load", [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(sc.Tuning)],
         ctypes.c_int),
        ("hl_tuning_parse", [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    ]:
        f = getattr(H, name)
        f.argtypes, f.restype = args, res
    return H


# ---- the C ABI ---------------------------------------------------------------

def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SPARKCL_API\s+[\w\s\*]+?\b(sparkcl_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(sc.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", libbuild.LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted(set(re.findall(r" T (sparkcl_\w+)", out)))
    assert exported == names  # nothing else leaks from the library


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include "sparkcl.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
                   "sizeof(sparkcl_task), sizeof(sparkcl_result), sizeof(sparkcl_config),"
                   "sizeof(sparkcl_tuning), sizeof(sparkcl_serve_stats), sizeof(sparkcl_launch_shape),"
                   "offsetof(sparkcl_task, coef), offsetof(sparkcl_result, t_done_ns),"
                   "offsetof(sparkcl_config, tune_cache));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src),
                           "-o", str(exe)])
    got = list(map(int, subprocess.check_output([str(exe)]).split()))
    want = [ctypes.sizeof(sc.Task), ctypes.sizeof(sc.Result), ctypes.sizeof(sc.Config),
            ctypes.sizeof(sc.Tuning), ctypes.sizeof(sc.ServeStats),
            ctypes.sizeof(sc.LaunchShape), sc.Task.coef.offset,
            sc.Result.t_done_ns.offset, sc.Config.tune_cache.offset]
    assert got == want


def test_strerror_and_version(lib):
    assert sc.strerror(sc.ETOOBIG) == "task too big"
    assert sc.strerror(sc.OK) == "ok"
    assert sc.version().startswith("sparkcl")


def test_init_fails_cleanly_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p(123)
    cfg = sc.Config()
    rc = lib.sparkcl_init(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == sc.EHIP and h.value is None
    assert b"device" in lib.sparkcl_last_error()
    assert lib.sparkcl_init(None, ctypes.byref(h)) == sc.EINVAL
    # calls on a null context are rejected, not crashed
    assert lib.sparkcl_reduce(None, None, 0, 0, None, None, None) == sc.EINVAL
    assert lib.sparkcl_poll(None, 1, None) == sc.EINVAL


def test_binding_fails_loudly_when_library_missing(monkeypatch, tmp_path):
    import paper_1505_01120_amd.sparkcl as mod
    monkeypatch.setattr(mod, "_lib", None)
    monkeypatch.setattr(mod, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        mod.load()


# ---- arena -------------------------------------------------------------------

def test_arena_alignment_and_coalescing(host):
    a = host.hl_arena_new(1 << 20)
    try:
        offs = [host.hl_arena_alloc(a, n) for n in (1, 255, 256, 257, 1000)]
        assert all(o % 256 == 0 for o in offs)
        assert offs == [0, 256, 512, 768, 1280]
        assert host.hl_arena_in_use(a) == 256 * 3 + 512 + 1024
        for o in (offs[1], offs[3], offs[2]):  # free the middle run out of order
            assert host.hl_arena_release(a, o) == 1
        assert host.hl_arena_release(a, offs[2]) == 0  # double free is refused
        assert host.hl_arena_alloc(a, 768) == 256      # coalesced hole is reused
        for o in (offs[0], 256, offs[4]):
            host.hl_arena_release(a, o)
        assert host.hl_arena_in_use(a) == 0 and host.hl_arena_free_blocks(a) == 1
        assert host.hl_arena_largest_free(a) == 1 << 20
        assert host.hl_arena_alloc(a, (1 << 20) + 1) == 2 ** 64 - 1
    finally:
        host.hl_arena_free(a)


def test_arena_random_against_model(host, datagen):
    size = 1 << 24
    a = host.hl_arena_new(size)
    w = datagen.fill(4000, 3, 0, 1, datagen.WORDS)
    live = {}
    try:
        for v in map(int, w):
            if live and v % 3 == 0:
                off = sorted(live)[v % len(live)]
                assert host.hl_arena_release(a, off) == 1
                del live[off]
            else:
                n = 1 + (v >> 8) % 200_000
                off = host.hl_arena_alloc(a, n)
                if off == 2 ** 64 - 1:
                    assert sum(live.values()) + n > 0  # failure only when fragmented/full
                    continue
                rounded = (n + 255) // 256 * 256
                for o, l in live.items():  # no overlap with any live block
                    assert off + rounded <= o or o + l <= off
                assert off + rounded <= size
                live[off] = rounded
            assert host.hl_arena_in_use(a) == sum(live.values())
        for off in list(live):
            host.hl_arena_release(a, off)
        assert host.hl_arena_free_blocks(a) == 1 and host.hl_arena_in_use(a) == 0
    finally:
        host.hl_arena_free(a)


# ---- admission ---------------------------------------------------------------

def admit(host, b):
    seq, slot, tk = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64()
    if not host.hl_adm_admit(b, ctypes.byref(seq), ctypes.byref(slot), ctypes.byref(tk)):
        return None
    return seq.value, slot.value, tk.value


def test_admission_budget_fifo_and_peak(host):
    b = host.hl_adm_new(1000, 8, 1 << 20)
    try:
        assert host.hl_adm_fits(b, 1000, 1) and not host.hl_adm_fits(b, 1001, 1)
        for t, nbytes in enumerate([400, 400, 300, 100], start=1):
            host.hl_adm_push(b, t, nbytes, 1, 0)
        assert admit(host, b) == (0, 0, 1)
        assert admit(host, b) == (1, 1, 2)
        assert host.hl_adm_head_block(b) == 3      # 300 more exceeds 1000
        assert admit(host, b) is None              # FIFO: the 100 behind it waits too
        assert host.hl_adm_complete(b, 0) == 1
        assert admit(host, b) == (2, 2, 3) and admit(host, b) == (3, 3, 4)
        assert host.hl_adm_peak(b) <= 1000 and host.hl_adm_in_use(b) == 800
        assert host.hl_adm_head_block(b) == 1      # empty
    finally:
        host.hl_adm_free(b)


def test_admission_slots_wrap(host):
    b = host.hl_adm_new(1 << 40, 4, 1 << 20)
    try:
        for t in range(6):
            host.hl_adm_push(b, t + 1, 1, 1, 0)
        got = [admit(host, b) for _ in range(4)]
        assert [g[1] for g in got] == [0, 1, 2, 3]
        assert host.hl_adm_head_block(b) == 2      # seq 4 maps to busy slot 0
        host.hl_adm_complete(b, 1)                 # slot 1 frees, but seq 4 needs 0
        assert admit(host, b) is None
        host.hl_adm_complete(b, 0)
        assert admit(host, b) == (4, 0, 5)
        assert host.hl_adm_head_block(b) == 0 and admit(host, b) == (5, 1, 6)
    finally:
        host.hl_adm_free(b)


def test_admission_tiles_and_unadmit(host):
    b = host.hl_adm_new(1 << 40, 64, 100)
    try:
        assert not host.hl_adm_fits(b, 1, 101)
        host.hl_adm_push(b, 1, 10, 60, 0)
        host.hl_adm_push(b, 2, 10, 60, 0)
        a1 = admit(host, b)
        assert host.hl_adm_head_block(b) == 4      # tile map full
        host.hl_adm_complete(b, a1[0])
        a2 = admit(host, b)
        assert a2 == (1, 1, 2) and host.hl_adm_tiles(b) == 60
        assert host.hl_adm_unadmit(b, a2[0]) == 1  # resources unavailable: back to queue
        assert host.hl_adm_pending(b) == 1 and host.hl_adm_in_flight(b) == 0
        assert admit(host, b) == (1, 1, 2)         # same sequence number again
    finally:
        host.hl_adm_free(b)


def take_slot(host, b, ticket):
    seq, slot = ctypes.c_uint64(), ctypes.c_uint32()
    if not host.hl_adm_take_slot(b, ticket, ctypes.byref(seq), ctypes.byref(slot)):
        return None
    return seq.value, slot.value


NO_SEQ = (1 << 64) - 1


def test_admission_staged_tasks_take_slots_when_ready(host):
    """A staged (host-input) task is admitted against the budget without a
    ring slot; it takes the next slot only once its inputs are on the device,
    so tasks admitted after it are not held up while it copies."""
    b = host.hl_adm_new(1000, 2, 1 << 20)
    try:
        host.hl_adm_push_staged(b, 1, 300, 1, 0)
        host.hl_adm_push(b, 2, 300, 1, 0)
        host.hl_adm_push(b, 3, 300, 1, 0)
        host.hl_adm_push_staged(b, 4, 200, 1, 0)
        assert admit(host, b) == (NO_SEQ, 0, 1)    # staged: charged, no slot
        assert admit(host, b) == (0, 0, 2)         # the device task goes first in the ring
        assert admit(host, b) == (1, 1, 3)
        assert host.hl_adm_in_use(b) == 900 and host.hl_adm_head_block(b) == 3  # budget
        assert take_slot(host, b, 1) is None       # ring full: both slots busy
        assert host.hl_adm_complete(b, 0) == 1
        assert take_slot(host, b, 1) == (2, 0)     # copied: takes the next slot
        assert take_slot(host, b, 1) is None       # not staged any more
        assert admit(host, b) == (NO_SEQ, 0, 4)    # a staged head ignores busy slots
        assert host.hl_adm_in_use(b) == 800
        assert host.hl_adm_unadmit_staged(b, 4) == 1   # no staging room: back to the queue
        assert host.hl_adm_pending(b) == 1 and host.hl_adm_in_use(b) == 600
        assert admit(host, b) == (NO_SEQ, 0, 4)
        assert host.hl_adm_complete_staged(b, 4) == 1  # failed before it took a slot
        assert host.hl_adm_complete_staged(b, 4) == 0
        assert host.hl_adm_in_flight(b) == 2 and host.hl_adm_in_use(b) == 600
        assert host.hl_adm_complete(b, 1) == 1 and host.hl_adm_complete(b, 2) == 1
        assert host.hl_adm_in_use(b) == 0 and host.hl_adm_in_flight(b) == 0
    finally:
        host.hl_adm_free(b)


# ---- tuning table ---------------------------------------------------------------

def test_tuning_defaults_valid_and_lookup(host):
    t = sc.Tuning()
    host.hl_tuning_defaults(ctypes.byref(t))
    assert host.hl_tuning_validate(ctypes.byref(t)) == 0
    assert [host.hl_size_bucket(n) for n in (0, 1, 2, 3, 1023, 1024, 1 << 22, (1 << 22) + 5)] == \
        [0, 0, 1, 1, 9, 10, 22, 22]
    assert host.hl_size_bucket(1 << 40) == 31
    for mode in range(3):
        for kid in (1, 2, 3):
            for n in (1, 1000, 1 << 16, 1 << 22, 1 << 30):
                T = host.hl_tile_for(ctypes.byref(t), mode, kid, n)
                assert T & (T - 1) == 0 and 1 << 10 <= T <= 1 << 22
    t.tile[1][0][5] = 3000
    assert host.hl_tuning_validate(ctypes.byref(t)) == sc.EINVAL


def test_tuning_json_roundtrip(host, tmp_path):
    t = sc.Tuning()
    host.hl_tuning_defaults(ctypes.byref(t))
    t.blocks_per_cu[0], t.blocks_per_cu[1], t.blocks_per_cu[2] = 1, 2, 7
    t.tile_many[0], t.tile_many[1] = 1 << 16, 1 << 17
    t.tile[1][1][22] = 1 << 16
    path = str(tmp_path / "tune.json").encode()
    assert host.hl_tuning_save(path, b"gfx950:sramecc+:xnack-", ctypes.byref(t)) == 1
    other = sc.Tuning()
    host.hl_tuning_defaults(ctypes.byref(other))
    assert host.hl_tuning_save(path, b"gfx942", ctypes.byref(other)) == 1  # kept side by side
    back = sc.Tuning()
    assert host.hl_tuning_load(path, b"gfx950:sramecc+:xnack-", ctypes.byref(back)) == 1
    assert bytes(back) == bytes(t)
    assert host.hl_tuning_load(path, b"gfx942", ctypes.byref(back)) == 1
    assert bytes(back) == bytes(other)
    assert host.hl_tuning_load(path, b"gfx1100", ctypes.byref(back)) == 0
    err = ctypes.create_string_buffer(256)
    assert host.hl_tuning_parse(open(path).read().encode(), err, 256) == 2
    bad = b'{"gfx950": {"tile": {"batched": {"poly": [1, 2]}}}}'
    assert host.hl_tuning_parse(bad, err, 256) == -1 and b"32 sizes" in err.value
    # a single number sets every kernel's occupancy
    assert host.hl_tuning_parse(b'{"gfx950": {"blocks_per_cu": 3}}', err, 256) == 1
    assert host.hl_tuning_parse(b'{"gfx950": {"blocks_per_cu": 40}}', err, 256) == -1
    assert host.hl_tuning_parse(b'{"gfx950": [}', err, 256) == -1
    # mixed-batch tiles: three entries, each 0 or a power of two in range
    assert host.hl_tuning_parse(b'{"gfx950": {"tile_many": [0, 65536, 0]}}', err, 256) == 1
    assert host.hl_tuning_parse(b'{"gfx950": {"tile_many": [0, 65536]}}', err, 256) == -1
    assert host.hl_tuning_parse(b'{"gfx950": {"tile_many": [0, 3000, 0]}}', err, 256) == -1
    assert b"tile_many" in err.value
    # block sizes (0 = default, 256, 512, 1024) and loads in flight (0, 2, 4, 8)
    assert host.hl_tuning_parse(b'{"gfx950": {"block": [512, 0, 1024], "block_many": 256,'
                                b' "unroll": [2, 8, 0]}}', err, 256) == 1
    for bad in (b'{"gfx950": {"block": [384, 0, 0]}}', b'{"gfx950": {"block": [256, 256]}}',
                b'{"gfx950": {"block_many": 2048}}', b'{"gfx950": {"unroll": [3, 4, 4]}}',
                b'{"gfx950": {"unroll": [16, 4, 4]}}'):
        assert host.hl_tuning_parse(bad, err, 256) == -1, bad
    t.block[0], t.block[2], t.block_many = 512, 1024, 1024
    t.unroll[0], t.unroll[1] = 8, 2
    assert host.hl_tuning_validate(ctypes.byref(t)) == 0
    assert host.hl_tuning_save(path, b"gfx950:sramecc+:xnack-", ctypes.byref(t)) == 1
    assert host.hl_tuning_load(path, b"gfx950:sramecc+:xnack-", ctypes.byref(back)) == 1
    assert bytes(back) == bytes(t)
    t.many_tiles_per_cu[0], t.many_tiles_per_cu[1] = 24, 4096
    t.blocks_per_cu_mc_only = 6
    assert host.hl_tuning_save(path, b"gfx950:sramecc+:xnack-", ctypes.byref(t)) == 1
    assert host.hl_tuning_load(path, b"gfx950:sramecc+:xnack-", ctypes.byref(back)) == 1
    assert bytes(back) == bytes(t) and list(back.many_tiles_per_cu) == [24, 4096]
    assert back.blocks_per_cu_mc_only == 6
    assert host.hl_tuning_parse(b'{"gfx950": {"blocks_per_cu_mc_only": 33}}', err, 256) == -1
    assert host.hl_tuning_parse(b'{"gfx950": {"many_tiles_per_cu": [8, 0]}}', err, 256) == 1
    for bad in (b'{"gfx950": {"many_tiles_per_cu": [8]}}',
                b'{"gfx950": {"many_tiles_per_cu": [4097, 8]}}'):
        assert host.hl_tuning_parse(bad, err, 256) == -1, bad
    t.unroll[2] = 5
    assert host.hl_tuning_validate(ctypes.byref(t)) == sc.EINVAL


def test_committed_tuning_cache_is_valid(host):
    path = sc.TUNING_PATH
    if not os.path.exists(path):
        pytest.skip("no tuning cache committed yet")
    err = ctypes.create_string_buffer(256)
    assert host.hl_tuning_parse(open(path).read().encode(), err, 256) >= 1, err.value


def test_hot_kernels_keep_registers_and_no_scratch():
    """The hot kernels stay inlined and in registers: no private segment (a
    non-inlined call or a spill puts state in scratch), at most 128 VGPRs
    (four waves per SIMD), and the Philox loop at its expected size.  Figures
    come from the device assembly of the current build."""
    if not os.path.exists(libbuild.ISA_JSON):
        libbuild.build()
    with open(libbuild.ISA_JSON) as f:
        isa = json.load(f)
    with open(os.path.join(libbuild.CSRC, "kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if isa.get("kernels_sha256_16") != sha:
        libbuild.build()
        with open(libbuild.ISA_JSON) as f:
            isa = json.load(f)
    # the wide array reduce holds a 7-level counter for 4 float4 columns per
    # thread and runs at three waves per SIMD (at most 168 VGPRs); so may the
    # chain executor's 8-loads instance, which short chains run at one block
    # (one wave per SIMD) per CU
    limit = {"k_tree_wide": 168, "k_chain": 168}
    for k in libbuild.KERNELS:
        assert isa[k]["private_segment_bytes"] == 0, (k, isa[k])
        assert isa[k]["vgpr_spills"] == 0, (k, isa[k])
        assert isa[k]["vgpr"] <= limit.get(k, 128), (k, isa[k])
    loop = isa["philox_loop"]
    # ten rounds of two 32x32->64 products and two three-way xors per lane
    assert loop["xor3"] == 20 and loop["mad_u64_u32"] >= 20, loop
    assert loop["valu"] < 70, loop


def test_header_constants_match_the_binding():
    """Every numeric #define of the C header that the Python binding also
    names (without the SPARKCL_ prefix) has the same value there."""
    with open(HEADER) as f:
        text = f.read()
    seen = {}
    for name, val in re.findall(r"^#define SPARKCL_(\w+)\s+\(?(-?\d+)u?\)?", text, re.M):
        seen[name] = int(val)
    for name in ("PER_LAUNCH", "BATCHED", "GRAPH", "POLY", "FMUL", "MC_PI", "SUM", "MAX",
                 "COUNT", "VADD", "VMAX", "TASK_HOST_INPUT", "FLAG_SERVE_PER_TASK", "OK",
                 "EINVAL", "EDECLINED", "TUNE_BUCKETS", "TUNE_MODES"):
        assert name in seen, name
    for name, val in seen.items():
        if hasattr(sc, name):
            assert getattr(sc, name) == val, (name, getattr(sc, name), val)


def test_load_generator_library_exports_one_entry(lib):
    """The serving load generator is its own library on top of the C ABI:
    one exported entry point, refusing bad arguments without a GPU."""
    if not os.path.exists(libbuild.LOADGEN_LIB):
        libbuild.build()
    out = subprocess.run(["nm", "-D", "--defined-only", libbuild.LOADGEN_LIB],
                         capture_output=True, text=True, check=True).stdout
    assert sorted(set(re.findall(r" T (\w+)", out))) == ["sparkcl_loadgen_run"]
    lg = ctypes.CDLL(libbuild.LOADGEN_LIB)
    t0 = ctypes.c_int64()
    assert lg.sparkcl_loadgen_run(None, None, None, ctypes.c_uint64(0), ctypes.c_int64(0),
                                  ctypes.c_uint32(0), ctypes.byref(t0), None, None,
                                  None) == sc.EINVAL


def test_probe_library_exports_and_refuses(lib):
    """The measurement probes are a library of their own, outside the API:
    the read ceiling, the VALU ceiling and the clock rates, each refusing bad
    arguments before any HIP call."""
    if not os.path.exists(libbuild.PROBE_LIB):
        libbuild.build()
    out = subprocess.run(["nm", "-D", "--defined-only", libbuild.PROBE_LIB],
                         capture_output=True, text=True, check=True).stdout
    assert sorted(set(re.findall(r" T (\w+)", out))) == [
        "sparkcl_probe_clock_rates", "sparkcl_probe_read2", "sparkcl_probe_valu"]
    pv = ctypes.CDLL(libbuild.PROBE_LIB).sparkcl_probe_valu
    pv.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert pv(0, 1, 1, 0, 0, None, 64, None) == sc.EINVAL       # no sink
    assert pv(0, 1, 1, 0, 0, 64, None, None) == sc.EINVAL       # no clock words
    assert pv(0, 0, 1, 0, 0, 64, 64, None) == sc.EINVAL         # empty grid
    assert pv(0, 1, 0, 0, 0, 64, 64, None) == sc.EINVAL         # no iterations
    assert pv(8, 1, 1, 0, 0, 64, 64, None) == sc.EINVAL         # unknown mix
    assert pv(0, 1, 1, 0, 0, 66, 64, None) == sc.EINVAL         # sink misaligned
    assert pv(0, 1, 1, 0, 0, 64, 68, None) == sc.EINVAL         # clock words misaligned
    cr = ctypes.CDLL(libbuild.PROBE_LIB).sparkcl_probe_clock_rates
    assert cr(0, None, None) == sc.EINVAL
    pr = ctypes.CDLL(libbuild.PROBE_LIB)
    fn = pr.sparkcl_probe_read2
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                   ctypes.c_void_p, ctypes.c_void_p]
    assert fn(None, None, 4096, 1, None, None) == sc.EINVAL
    # 16-byte aligned stand-ins that are never dereferenced: every call below
    # fails its size or alignment check first
    assert fn(16, 32, 4096, 0, 64, None) == sc.EINVAL          # empty grid
    assert fn(16, 32, 4095, 1, 64, None) == sc.EINVAL          # n not a whole pass
    assert fn(16, 32, 4096 * 3, 2, 64, None) == sc.EINVAL      # 1.5 passes of 2 blocks
    assert fn(20, 32, 4096, 1, 64, None) == sc.EINVAL          # x not 16-byte aligned
