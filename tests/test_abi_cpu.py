"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/ps.h, and rejects bad arguments before launching
anything (every call below returns from argument checking, so no HIP call
is made)."""

import ctypes
import itertools
import math

import pytest

ps = pytest.importorskip("paper_1705_08210_amd.ps")
lib = ps.lib

FAKE = ctypes.c_void_p(0x10000)   # never dereferenced: calls fail before use
OK, ARG, DTYPE, WS, HIP, UNSUP = range(6)


def test_exports_every_declared_function():
    names = ps.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _header_enums():
    """name -> value of every enumerator and #define alias in include/ps.h."""
    import re
    txt = re.sub(r"/\*.*?\*/", "", open(ps.HEADER).read(), flags=re.S)
    vals = {m.group(1): int(m.group(2))
            for m in re.finditer(r"\b(PS_[A-Z0-9_]+)\s*=\s*(\d+)", txt)}
    for m in re.finditer(r"#define\s+(PS_[A-Z0-9_]+)\s+(PS_[A-Z0-9_]+)", txt):
        vals[m.group(1)] = vals[m.group(2)]
    return vals


def test_enum_values_match_the_boundary():
    """The numbering of the status, storage, accumulation and path enums,
    as the header declares them and as the binding passes them."""
    v = _header_enums()
    assert [v[n] for n in ("PS_OK", "PS_ERR_ARG", "PS_ERR_DTYPE", "PS_ERR_WORKSPACE",
                           "PS_ERR_HIP", "PS_ERR_UNSUPPORTED")] == [0, 1, 2, 3, 4, 5]
    assert [v[n] for n in ("PS_F32", "PS_F16", "PS_U8", "PS_F64")] == [0, 1, 2, 3]
    assert [v[n] for n in ("PS_ACC_PLAIN", "PS_ACC_BLOCKED", "PS_ACC_AUTO")] == [0, 1, 2]
    assert [v[n] for n in ("PS_PATH_AUTO", "PS_PATH_VALU", "PS_PATH_MFMA",
                           "PS_PATH_MFMA_FP4", "PS_PATH_BITS")] == [0, 1, 2, 3, 4]
    assert v["PS_PATH_MFMA_THERMO"] == v["PS_PATH_MFMA"]
    assert ps.ACC == {"plain": 0, "blocked": 1, "auto": 2}
    assert ps.PATH == {"auto": 0, "valu": 1, "mfma": 2, "mfma_fp4": 3, "bits": 4}
    assert (ps.PS_F32, ps.PS_F16, ps.PS_U8, ps.PS_F64) == (0, 1, 2, 3)


def test_zero_filled_opts_mean_plain_accumulation():
    """A zero-filled ps_opts asks for PLAIN accumulation (no field-chunk
    partials); NULL opts mean AUTO (partials beyond 4096 fields)."""
    f = lib.ps2_workspace_size
    zero = ctypes.byref(ps.Opts(0, 0, 0, 0))
    assert f(0, 9000, 20000, 1, zero) == 0
    assert f(0, 9000, 20000, 1, None) > 0


def test_version_and_status_strings():
    assert lib.ps_version() == 10000
    for st, name in enumerate(["PS_OK", "PS_ERR_ARG", "PS_ERR_DTYPE", "PS_ERR_WORKSPACE",
                               "PS_ERR_HIP", "PS_ERR_UNSUPPORTED"]):
        assert lib.ps_status_string(st).decode() == name


def opts(acc=2, path=0, levels=0, tile=0):
    return ctypes.byref(ps.Opts(acc, path, levels, tile))


def call2(V=FAKE, dt=0, n_f=10, n_v=5, ld=10, s=None, c2=FAKE, n2=None, ws=FAKE,
          ws_bytes=1 << 20, o=None):
    return lib.ps2_compute(V, dt, n_f, n_v, ld, s, c2, n2, ws, ws_bytes, o, None)


@pytest.mark.parametrize("kw,status", [
    (dict(dt=7), DTYPE),
    (dict(n_f=-1), ARG),
    (dict(n_v=-3), ARG),
    (dict(ld=9), ARG),
    (dict(V=None), ARG),
    (dict(c2=None, n2=None), ARG),
    (dict(V=ctypes.c_void_p(0x10002)), ARG),           # not 4-byte aligned for FP32
    (dict(c2=ctypes.c_void_p(0x10001)), ARG),
    (dict(ws_bytes=16), WS),                           # sums need 256 bytes
    (dict(ws=None), WS),
    (dict(ws=ctypes.c_void_p(0x10010)), ARG),          # workspace not 256-aligned
    (dict(o=opts(acc=9)), ARG),
    (dict(o=opts(path=5)), ARG),
    (dict(o=opts(tile=99)), ARG),
    (dict(o=opts(levels=200)), ARG),
    (dict(o=opts(path=2)), UNSUP),                     # MFMA needs uint8 data
    (dict(dt=2, o=opts(path=2, levels=0)), ARG),       # MFMA needs levels
    (dict(o=opts(path=3, levels=3)), UNSUP),           # fp4 MFMA needs uint8 data
    (dict(dt=2, n_f=6_000_000, ld=6_000_000, o=opts(path=3, levels=3)), ARG),  # > 2^24
    # int8 MFMA: 256 plane rows of 3 x 3M bytes exceed 32-bit tile offsets
    # int8 planes (levels * n_f >= 2^24): 256 plane rows past 2^31 bytes
    (dict(dt=2, n_f=3_000_000, ld=3_000_000, o=opts(path=2, levels=15)), UNSUP),
    # fused int8 (levels * n_f < 2^24): 256 rows of V past 2^31 bytes
    (dict(dt=2, n_f=1000, ld=9_000_000, o=opts(path=2, levels=3)), UNSUP),
    (dict(o=opts(path=4)), UNSUP),                     # bits need uint8 data
    (dict(dt=2, o=opts(path=4, levels=0)), ARG),       # bits need levels = 1
    (dict(dt=2, o=opts(path=4, levels=2)), ARG),
    (dict(o=opts(path=5)), ARG),
])
def test_ps2_argument_errors(kw, status):
    assert call2(**kw) == status
    assert lib.ps_last_error().decode() != ""


BIG_NF = 8_421_505          # 255 * n_f >= 2^31: the uint8 VALU sums would overflow


@pytest.mark.parametrize("o", [None, opts(path=1), opts(path=1, levels=3)])
def test_u8_valu_rejects_fields_beyond_its_integer_range(o):
    assert call2(dt=2, n_f=BIG_NF, ld=BIG_NF, o=o) == UNSUP
    assert "uint8 VALU" in lib.ps_last_error().decode()
    assert call3(dt=2, n_f=BIG_NF, ld=BIG_NF, o=o) == UNSUP
    # one field fewer is inside the range (it fails later, at the fake workspace)
    assert call2(dt=2, n_f=BIG_NF - 1, ld=BIG_NF, ws_bytes=16, o=o) == WS


def test_u8_valu_range_in_a_batch():
    arr = (ps.Problem * 2)()
    arr[0] = ps.Problem(FAKE, 10, 5, 10, None, FAKE, None)
    arr[1] = ps.Problem(FAKE, BIG_NF, 5, BIG_NF, None, FAKE, None)
    assert lib.ps2_compute_batched(arr, 2, 2, FAKE, 1 << 20, None, None) == UNSUP
    assert "problem 1" in lib.ps_last_error().decode()
    # floating data has no such bound
    assert lib.ps2_compute_batched(arr, 2, 0, FAKE, 16, None, None) == WS


def call2s(shard, nshards, **kw):
    """ps2_compute_shard with call2's fake arguments."""
    a = dict(V=FAKE, dt=0, n_f=10, n_v=5, ld=10, s=None, c2=FAKE, n2=None, ws=FAKE,
             ws_bytes=1 << 20, o=None)
    a.update(kw)
    return lib.ps2_compute_shard(a["V"], a["dt"], a["n_f"], a["n_v"], a["ld"], a["s"],
                                 a["c2"], a["n2"], shard, nshards, a["ws"], a["ws_bytes"],
                                 a["o"], None)


@pytest.mark.parametrize("shard,nshards,kw,status", [
    (0, 0, {}, ARG),                                   # no shards
    (-1, 4, {}, ARG),
    (4, 4, {}, ARG),                                   # shard past the last
    (1, 4, dict(dt=2, o=opts(path=2, levels=3)), UNSUP),   # MFMA paths are not sharded
    (1, 4, dict(ws_bytes=16), WS),                     # arguments fine up to the workspace
    (1, 4, dict(o=opts(acc=1), ws_bytes=16), WS),      # BLOCKED: chunk partials in the workspace
    (0, 1, dict(o=opts(acc=1), ws_bytes=16), WS),      # one shard is ps2_compute
])
def test_ps2_shard_argument_errors(shard, nshards, kw, status):
    assert call2s(shard, nshards, **kw) == status


def test_ps2_no_pairs_is_noop():
    # n_v < 2: nothing to compute, nothing launched, pointers unused
    assert call2(n_v=1, c2=None, ws=None, ws_bytes=0) == OK
    assert call2(n_v=0, c2=None, V=None, ws=None, ws_bytes=0) == OK


def test_sums_argument_errors():
    f = lib.ps_vector_sums
    assert f(FAKE, 9, 10, 5, 10, FAKE, None, None) == DTYPE
    assert f(FAKE, 0, 10, 5, 10, None, None, None) == ARG
    assert f(FAKE, 0, 10, 5, 3, FAKE, None, None) == ARG
    assert f(FAKE, 0, 10, 5, 10, ctypes.c_void_p(0x10004), None, None) == ARG
    assert f(FAKE, 0, 10, 5, 10, FAKE, ctypes.c_void_p(0x10002), None) == ARG


def call3(V=FAKE, dt=0, n_f=10, n_v=6, ld=10, s=None, n2=None, jb=1, je=5, c3=FAKE,
          ws=FAKE, ws_bytes=1 << 20, o=None):
    return lib.ps3_compute(V, dt, n_f, n_v, ld, s, n2, jb, je, c3, ws, ws_bytes, o, None)


@pytest.mark.parametrize("kw,status", [
    (dict(jb=0), ARG),
    (dict(je=6), ARG),
    (dict(jb=4, je=3), ARG),
    (dict(c3=None), ARG),
    (dict(ws_bytes=100), WS),
    (dict(dt=5), DTYPE),
    (dict(o=opts(path=2)), UNSUP),
    (dict(o=opts(path=4, levels=1)), UNSUP),           # bits need uint8 data
    (dict(dt=2, o=opts(path=4, levels=3)), ARG),
    (dict(dt=2, o=opts(path=2, levels=0)), ARG),       # MFMA needs levels
    (dict(dt=2, n_f=6_000_000, ld=6_000_000, o=opts(path=3, levels=3)), ARG),  # > 2^24
    # int8 planes (levels * n_f >= 2^24): 256 plane rows past 2^31 bytes
    (dict(dt=2, n_f=3_000_000, ld=3_000_000, o=opts(path=2, levels=15)), UNSUP),
    # fused int8 (levels * n_f < 2^24): 256 rows of V past 2^31 bytes
    (dict(dt=2, n_f=1000, ld=9_000_000, o=opts(path=2, levels=3)), UNSUP),
])
def test_ps3_argument_errors(kw, status):
    assert call3(**kw) == status


def call3_noalloc(V=FAKE, dt=0, n_f=10, n_v=6, ld=10, s=None, n2=None, jb=1, je=5, c3=FAKE,
                  o=None):
    return lib.ps3_compute_noalloc(V, dt, n_f, n_v, ld, s, n2, jb, je, c3, o, None)


@pytest.mark.parametrize("kw,status", [
    (dict(jb=0), ARG),
    (dict(jb=4, je=3), ARG),
    (dict(c3=None), ARG),
    (dict(dt=5), DTYPE),
    (dict(o=opts(path=2)), UNSUP),
    (dict(dt=2, o=opts(path=2, levels=0)), ARG),
    # the pair table of 4200 vectors (35 MB) does not fit the static scratch
    (dict(n_f=8, ld=8, n_v=4200, je=2), WS),
])
def test_ps3_noalloc_argument_errors(kw, status):
    """Checked before the static scratch is looked up, so no HIP call."""
    assert call3_noalloc(**kw) == status


def test_noalloc_scratch_size_is_the_header_constant():
    assert ps.noalloc_scratch_bytes() == 32 << 20
    g = lib.ps3_workspace_size
    assert g(0, 8, 4200, 0, 0, 1, 2, None) > ps.noalloc_scratch_bytes()
    assert call3_noalloc(n_f=8, ld=8, n_v=4200, je=2) == WS
    assert "static scratch" in lib.ps_last_error().decode()
    assert call3_noalloc(jb=3, je=3, c3=None) == OK        # empty stage: nothing to do


def test_ps3_empty_cases_are_noops():
    assert call3(jb=3, je=3, c3=None, ws=None, ws_bytes=0) == OK
    assert call3(n_v=2, jb=1, je=1, c3=None, ws=None, ws_bytes=0) == OK


def test_workspace_sizes():
    f = lib.ps2_workspace_size
    assert f(0, 100, 1000, 0, None) == 8192        # n_v doubles, 256-aligned
    assert f(0, 100, 1000, 1, None) == 0
    g = lib.ps3_workspace_size
    n = 100
    pairs = n * (n - 1) // 2
    prefixes = math.ceil(2 * (n + 1) * 8 / 256) * 256    # whole-tile and edge-tile slab prefixes
    expect = math.ceil(n * 8 / 256) * 256 + math.ceil(pairs * 4 / 256) * 256 + prefixes
    assert g(0, 10, n, 0, 0, 1, n - 1, None) == expect
    assert g(0, 10, n, 1, 1, 1, n - 1, None) == prefixes
    # blocked accumulation beyond 4096 fields: FP32 partials of each field chunk
    stage = math.comb(n, 3)
    assert g(0, 9000, n, 1, 1, 1, n - 1, None) == prefixes + math.ceil(3 * stage * 4 / 256) * 256
    blocked = opts(acc=1)
    assert f(0, 9000, 1000, 1, blocked) == math.ceil(3 * (1000 * 999 // 2) * 4 / 256) * 256
    assert f(0, 9000, 1000, 1, opts(acc=0)) == 0   # plain: one chunk, no partials
    # auto on a small triangle splits further so that enough workgroups run
    assert f(0, 9000, 1000, 1, None) > f(0, 9000, 1000, 1, blocked)
    assert f(2, 9000, 1000, 1, None) == 0          # integer data: no split
    # bits: the packed matrix, 32 fields per word in whole 16-byte chunks
    words = math.ceil(math.ceil(9000 / 32) / 4) * 4
    assert f(2, 9000, 1000, 1, opts(path=4, levels=1)) == math.ceil(1000 * words * 4 / 256) * 256
    # auto with levels 1..15: the int8 MFMA path thresholds V's bytes in
    # registers, no plane workspace; the 4x4 wave layout (tile 2) and fp4 read
    # planes (3 levels x 1024 padded fields per vector, 2 fields per byte for fp4)
    assert f(2, 1000, 1000, 1, opts(levels=3)) == 0
    assert f(2, 1000, 1000, 1, opts(path=2, levels=3, tile=2)) == \
        math.ceil(1000 * 3 * 1024 / 256) * 256
    assert f(2, 1000, 1000, 1, opts(path=3, levels=3)) == \
        math.ceil(1000 * 3 * 1024 / 2 / 256) * 256
    # more than 7 levels with levels * n_f >= 2^24: int8 planes, unless 256
    # plane rows exceed 32-bit offsets (then AUTO takes the VALU path)
    assert f(2, 6_000_000, 100, 1, opts(path=2, levels=9)) == \
        100 * 9 * math.ceil(6_000_000 / 128) * 128
    assert f(2, 6_000_000, 100, 1, opts(path=2, levels=7)) == 0   # counts up to 2^31
    assert f(2, 3_000_000, 1000, 1, opts(levels=15)) == f(2, 3_000_000, 1000, 1,
                                                          opts(path=1, levels=3)) == 0


@pytest.mark.parametrize("n_v", [3, 4, 7, 20])
def test_stage_sizes_match_jslab_enumeration(n_v):
    """off(j) of the j-slab layout equals the count of triples with a smaller
    middle index, enumerated directly."""
    trip = [(i, j, k) for j in range(1, n_v - 1) for k in range(j + 1, n_v) for i in range(j)]
    assert lib.ps3_stage_size(n_v, 1, n_v - 1) == math.comb(n_v, 3) == len(trip)
    for jb, je in itertools.combinations(range(1, n_v), 2):
        cnt = sum(1 for t in trip if jb <= t[1] < je)
        assert lib.ps3_stage_size(n_v, jb, je) == cnt


def test_tile_configs_and_tuning_table():
    cfgs = ps.tile_configs()
    assert cfgs[0] == (128, 128, 32)
    assert (64, 64, 32) in cfgs
    import torch
    assert ps.tile_configs(torch.uint8)[0] == (128, 128, 128)     # 4 fields per word
    assert ps.tile_configs(torch.float16)[0] == (128, 128, 64)
    assert lib.ps_tune_register(0, 2, 1, 0, 10, 0, 10, 99) == ARG
    assert lib.ps_tune_register(0, 4, 1, 0, 10, 0, 10, 0) == ARG
    assert lib.ps_tune_register(0, 2, 1, 0, 10, 0, 10, 1) == OK
    # matrix-core tile orders (uint8, 2-way) and the AUTO path for integer levels
    assert lib.ps_tile_config(2, 2, 2, 0, None, None, None) == 5
    assert lib.ps_tile_config(2, 3, 2, 0, None, None, None) == 2   # 3-way tilings
    assert lib.ps_tile_config(0, 2, 3, 0, None, None, None) == 0
    assert lib.ps_tune_register(2, 2, 2, 0, 10, 0, 10, 4) == OK
    assert lib.ps_tune_register(2, 2, 2, 0, 10, 0, 10, 5) == ARG
    for code in (1, 2, 3):
        assert lib.ps_tune_register(2, 3, 0, 0, 10, 0, 10, code) == OK
    assert lib.ps_tune_register(2, 2, 0, 0, 10, 0, 10, 4) == ARG    # BITS is not a choice
    assert lib.ps_tune_register(0, 2, 0, 0, 10, 0, 10, 2) == ARG    # float data: no path choice
    lib.ps_tune_clear()


def test_tuned_auto_path_changes_the_workspace_query():
    """A registered AUTO choice of the VALU path for a uint8 shape removes
    the matrix-core path from the workspace query (AUTO with levels 1..15
    otherwise takes the int8 path; the fp4 choice needs its planes)."""
    f = lib.ps2_workspace_size
    o3 = opts(levels=3)
    base = f(2, 5000, 300, 1, o3)                 # int8 in registers: no planes
    assert base == 0
    assert lib.ps_tune_register(2, 2, 0, 0, 1 << 40, 0, 1 << 40, 3) == OK   # fp4
    assert f(2, 5000, 300, 1, o3) == math.ceil(300 * 3 * math.ceil(5000 / 256) * 128 / 256) * 256
    assert lib.ps_tune_register(2, 2, 0, 0, 1 << 40, 0, 1 << 40, 1) == OK   # VALU
    assert f(2, 5000, 300, 1, o3) == 0
    lib.ps_tune_clear()
    import paper_1705_08210_amd.autotune as at
    at.load()


def test_batched_argument_errors():
    arr = (ps.Problem * 2)()
    arr[0] = ps.Problem(FAKE, 10, 5, 10, None, FAKE, None)
    arr[1] = ps.Problem(FAKE, 10, 5, 9, None, FAKE, None)     # ld < n_f
    assert lib.ps2_compute_batched(arr, 2, 0, FAKE, 1 << 20, None, None) == ARG
    assert "problem 1" in lib.ps_last_error().decode()
    arr[1] = ps.Problem(FAKE, 10, 5, 10, None, None, None)    # no outputs
    assert lib.ps2_compute_batched(arr, 2, 0, FAKE, 1 << 20, None, None) == ARG
    arr[1] = ps.Problem(FAKE, 10, 5, 10, None, FAKE, None)
    assert lib.ps2_compute_batched(arr, 2, 0, FAKE, 16, None, None) == WS
    assert lib.ps2_compute_batched(arr, -1, 0, FAKE, 16, None, None) == ARG
    assert lib.ps2_compute_batched(arr, 0, 0, None, 0, None, None) == OK
    h = ctypes.c_void_p()
    assert lib.ps_plan_create_batched(None, arr, 2, 0, None, FAKE, 1 << 20, None) == ARG
    assert lib.ps_plan_create_batched(ctypes.byref(h), arr, 2, 0, None, FAKE, 16, None) == WS
    assert h.value is None
    assert lib.ps_plan_execute(None, None) == ARG
    lib.ps_plan_destroy(None)
