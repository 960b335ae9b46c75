"""2-way parity: the HIP path (through the C ABI) against the CPU oracle, on
seeded inputs that span several tiles with ragged tails, plus the exact
families and properties that hold at any size."""

import numpy as np
import pytest

import oracle
import workloads
from psx import (announce, check_exact_f32, check_rel, colex, host, need_gpu,
                 sample_pairs, to_dev)

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP16_TOL = 1e-3


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run2(V, **kw):
    from paper_1705_08210_amd import ps
    Vd = to_dev(V)
    c2, n2 = ps.ps2(Vd, want_n2=True, **kw)
    return host(c2), host(n2)


# ---------------------------------------------------------------- sums ----

@pytest.mark.parametrize("kind", ["f32", "f16", "u8"])
def test_sums_match_oracle(kind):
    from paper_1705_08210_amd import ps
    if kind == "u8":
        V = workloads.levels(301, 1003, seed=3)
    else:
        V = workloads.gwas_like(301, 1003, seed=3)
        if kind == "f16":
            V = workloads.to_f16(V)
    announce(f"sums {kind} {V.shape}")
    s, bad = ps.vector_sums(to_dev(V))
    s = host(s)
    ref = oracle.sums(V)
    if kind == "u8":
        assert np.array_equal(s, ref)
    else:
        check_rel(s, ref, 1e-13, "sums")
    assert host(bad)[0] == 0


def test_sums_count_out_of_domain_entries():
    from paper_1705_08210_amd import ps
    V = workloads.uniform(9, 77, seed=1)
    V[0, 5] = -1.0
    V[3, 0] = np.nan
    V[8, 76] = np.inf
    V[4, 4] = -0.0          # zero: in the domain
    announce("sums bad count")
    for dt in (np.float32, np.float16):
        _, bad = ps.vector_sums(to_dev(V.astype(dt)))
        assert host(bad)[0] == 3


# ------------------------------------------------------- oracle parity ----

def test_uniform_1024x256_full():
    V = workloads.uniform_1024x256()
    announce("2-way uniform 1024x256 full")
    c2, n2 = run2(V)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_rel(c2, ref, FP32_TOL, "c2")
    check_rel(n2, rn2, FP32_TOL, "n2")


@pytest.mark.parametrize("tile", [1, 2, 3])
@pytest.mark.parametrize("acc", ["plain", "blocked"])
def test_ragged_tiles_and_accumulation(tile, acc):
    V = workloads.gwas_like(300, 1001, seed=7)      # 3 tiles of 128 + tail; K tail
    announce(f"2-way ragged tile={tile} acc={acc}")
    c2, n2 = run2(V, tile=tile, acc=acc)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_rel(c2, ref, FP32_TOL, "c2")
    check_rel(n2, rn2, FP32_TOL, "n2")


@pytest.mark.parametrize("storage", ["f32", "u8"])
@pytest.mark.parametrize("tile", [1, 2, 3])
def test_integer_levels_bit_exact(storage, tile):
    V = workloads.levels(263, 777, seed=11)
    if storage == "f32":
        V = V.astype(np.float32)
    announce(f"2-way integer {storage} tile={tile}")
    c2, n2 = run2(V, tile=tile)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_exact_f32(c2, ref, "c2")
    assert np.array_equal(n2.astype(np.float64), rn2)


def test_fp16_storage():
    V32 = workloads.uniform(200, 1500, seed=5)
    V16 = workloads.to_f16(V32)
    announce("2-way fp16 storage")
    c2, n2 = run2(V16)
    # kernel error: against the oracle on the FP16-rounded values
    check_rel(c2, oracle.c2_all(V16), FP32_TOL, "c2 vs fp16 values")
    # user-visible error: against the FP32 source
    check_rel(c2, oracle.c2_all(V32), FP16_TOL, "c2 vs fp32 source")


@pytest.mark.parametrize("kind", ["f32", "f16", "u8"])
def test_unaligned_stride(kind):
    """Rows whose pitch is not a multiple of 16 bytes take the element-wise
    staging path."""
    import torch
    from paper_1705_08210_amd import ps
    n_v, n_f, ld = 150, 333, 337
    if kind == "u8":
        big = workloads.levels(n_v, ld, seed=2)
    else:
        big = workloads.sparse_uniform(n_v, ld, seed=2)
        if kind == "f16":
            big = workloads.to_f16(big)
    V = big[:, :n_f]
    announce(f"2-way unaligned {kind}")
    Vd = to_dev(big)[:, :n_f]
    assert Vd.stride(0) == ld
    c2, n2 = ps.ps2(Vd, want_n2=True)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    if kind == "u8":
        check_exact_f32(host(c2), ref, "c2")
    else:
        check_rel(host(c2), ref, FP32_TOL, "c2")
    del torch


@pytest.mark.parametrize("n_v,n_f", [(2, 1), (3, 5), (127, 31), (128, 32), (129, 33),
                                     (65, 1), (257, 7)])
def test_edge_sizes(n_v, n_f):
    V = workloads.sparse_uniform(n_v, n_f, seed=n_v + n_f)
    announce(f"2-way edge n_v={n_v} n_f={n_f}")
    c2, _ = run2(V)
    check_rel(c2, oracle.c2_all(V), FP32_TOL, "c2")


def test_zero_fields_and_zero_vectors():
    from paper_1705_08210_amd import ps
    import torch
    announce("2-way n_f=0 and zero vectors")
    V0 = torch.zeros((5, 0), dtype=torch.float32, device="cuda")
    c2, _ = ps.ps2(V0)
    assert np.all(host(c2) == 0)
    V = workloads.uniform(40, 50, seed=4)
    V[[3, 17, 18]] = 0.0
    c2, _ = run2(V)
    ref = oracle.c2_all(V)
    check_rel(c2, ref, FP32_TOL, "c2")
    assert c2[colex(17, 18)] == 0.0


def test_noop_sizes():
    from paper_1705_08210_amd import ps
    import torch
    for n_v in (0, 1):
        V = torch.rand((n_v, 10), device="cuda")
        c2, _ = ps.ps2(V)
        assert c2.numel() == 0


def test_given_sums_identical():
    from paper_1705_08210_amd import ps
    V = workloads.gwas_like(200, 900, seed=9)
    announce("2-way given sums")
    Vd = to_dev(V)
    s, _ = ps.vector_sums(Vd)
    a, _ = ps.ps2(Vd)
    b, _ = ps.ps2(Vd, s=s)
    assert np.array_equal(host(a), host(b))


def test_determinism_and_permutation_equivariance():
    """Each pair sums its fields in the same order whatever tile it lands
    in, so permuting the vectors permutes the outputs bit for bit."""
    V = workloads.gwas_like(300, 2100, seed=12)
    perm = np.random.default_rng(0).permutation(300)
    announce("2-way determinism/permutation")
    a, _ = run2(V)
    b, _ = run2(V)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    p, _ = run2(V[perm])
    i, j = np.triu_indices(300, 1)
    pi, pj = np.minimum(perm[i], perm[j]), np.maximum(perm[i], perm[j])
    assert np.array_equal(p[colex(i, j)].view(np.uint32), a[colex(pi, pj)].view(np.uint32))


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_nested_support_family_exact(storage):
    """V[perm(q), i] = a_i [q < L_i]: n2 = min(a) min(L), s_i = a_i L_i; all
    partial sums are exact dyadic values, so every path is bit-exact."""
    V, a, L = workloads.nested_support(390, 3000, seed=21, integer=(storage == "u8"))
    if storage == "f16":
        V = workloads.to_f16(V)
    announce(f"2-way nested support {storage}")
    c2, n2 = run2(V)
    i, j = np.triu_indices(len(a), 1)
    num = np.minimum(a[i], a[j]) * np.minimum(L[i], L[j])
    d = a[i] * L[i] + a[j] * L[j]
    ref = np.where(d > 0, 2 * num / np.where(d > 0, d, 1), 0.0)
    idx = colex(i, j)
    check_exact_f32(c2[idx], ref, "c2")
    assert np.array_equal(n2[idx].astype(np.float64), num)


def test_sampled_pairs_match_listed_oracle():
    V = workloads.gwas_like(700, 4000, seed=13)
    I, J = sample_pairs(700, 4000, seed=1)
    announce("2-way sampled pairs 700x4000")
    c2, _ = run2(V)
    check_rel(c2[colex(I, J)], oracle.c2_pairs(V, I, J), FP32_TOL, "c2 sampled")


# ------------------------------------------------ thermometer MFMA path ----

@pytest.mark.parametrize("wide", [0, 2])
@pytest.mark.parametrize("path", ["mfma", "mfma_fp4"])
@pytest.mark.parametrize("n_v,n_f,L", [(300, 1001, 3), (257, 64, 1), (513, 333, 7),
                                       (2, 5, 3), (256, 128, 3), (40, 3000, 15),
                                       (300, 1024, 3), (513, 320, 7), (41, 3008, 15),
                                       (1000, 192, 2), (300, 1008, 3), (257, 48, 1),
                                       (513, 2000, 7), (41, 16, 15), (300, 128, 4),
                                       (200, 256, 5), (130, 64, 6)])
def test_mfma_thermometer_bit_exact(n_v, n_f, L, path, wide):
    """min(a,b) = sum_t [a>=t][b>=t] on integer levels: the int8 matrix-core
    path must equal the oracle (and the VALU path) bit for bit."""
    probs = np.full(L + 1, 1.0 / (L + 1))
    V = workloads.levels(n_v, n_f, seed=n_v + L, probs=probs)
    announce(f"2-way {path} n_v={n_v} n_f={n_f} L={L} tile={wide}")
    c2, n2 = run2(V, path=path, levels=L, tile=wide)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_exact_f32(c2, ref, "c2")
    assert np.array_equal(n2.astype(np.float64), rn2)
    v2, vn2 = run2(V, path="valu")
    assert np.array_equal(c2.view(np.uint32), v2.view(np.uint32))
    assert np.array_equal(n2, vn2)


def test_mfma_auto_path_and_unaligned_rows():
    """levels in 1..15 selects the matrix-core path by default; rows whose
    pitch is not 16-byte aligned are expanded element by element."""
    from paper_1705_08210_amd import ps
    big = workloads.levels(200, 517, seed=41)
    V = big[:, :511]
    announce("2-way mfma auto + unaligned")
    Vd = to_dev(big)[:, :511]
    c2, _ = ps.ps2(Vd, levels=3)
    check_exact_f32(host(c2), oracle.c2_all(V), "c2")


def test_mfma_padded_rows_partial_last_stage():
    """Aligned rows (pitch 1024) whose length is not a multiple of the
    64-field stage take the register-staged tiles; the bytes past n_f (here
    255, inside the row pitch) must not count."""
    from paper_1705_08210_amd import ps
    for n_v, n_f, L in [(300, 1001, 3), (129, 77, 15)]:
        big = workloads.levels(n_v, 1024, seed=n_v + n_f, probs=np.full(L + 1, 1.0 / (L + 1)))
        big[:, n_f:] = 255
        V = np.ascontiguousarray(big[:, :n_f])
        announce(f"2-way mfma padded rows n_v={n_v} n_f={n_f} ld=1024 L={L}")
        Vd = to_dev(big)[:, :n_f]
        c2, n2 = ps.ps2(Vd, want_n2=True, path="mfma", levels=L)
        ref, rn2 = oracle.c2_all(V, with_n2=True)
        check_exact_f32(host(c2), ref, "c2")
        assert np.array_equal(host(n2).astype(np.float64), rn2)


def test_mfma_rows_beyond_32bit_tile_offsets():
    """Rows too long for 32-bit offsets over a 256-row tile: an explicit MFMA
    path is refused (PS_ERR_UNSUPPORTED) and AUTO takes the VALU path, still
    exact.  The int8 path that thresholds V in registers is bound by the row
    stride of V (256 ld < 2^31); with levels * n_f >= 2^24 it reads planes,
    bound by the plane-row length (256 levels kpad < 2^31)."""
    import torch
    from paper_1705_08210_amd import ps
    n_f = 2_900_000
    V = workloads.levels(3, n_f, seed=43)
    Vd = to_dev(V)
    ref = oracle.c2_all(V)
    announce(f"2-way mfma n_f={n_f} in registers")
    c2, _ = ps.ps2(Vd, path="mfma", levels=3)     # 3 n_f < 2^24, stride 2.9e6 fits
    check_exact_f32(host(c2), ref, "c2 int8 in registers")
    announce(f"2-way mfma planes limit n_f={n_f} levels=15")
    with pytest.raises(ps.PSError) as e:
        ps.ps2(Vd, path="mfma", levels=15)          # planes: 4.4e7 bytes per row
    assert e.value.status == 5
    c2, _ = ps.ps2(Vd, levels=15)
    check_exact_f32(host(c2), ref, "c2 auto levels=15")
    announce("2-way mfma stride limit ld=9e6")
    big = torch.zeros((3, 9_000_000), dtype=torch.uint8, device=Vd.device)
    big[:, :1000] = Vd[:, :1000]
    view = big[:, :1000]                            # n_f = 1000, ld = 9e6
    with pytest.raises(ps.PSError) as e:
        ps.ps2(view, path="mfma", levels=3)
    assert e.value.status == 5
    c2, _ = ps.ps2(view, levels=3)
    check_exact_f32(host(c2), oracle.c2_all(np.ascontiguousarray(V[:, :1000])), "c2 auto ld")


# ------------------------------------------ blocked (field-chunk) split ----

@pytest.mark.parametrize("tile", [1, 2, 3])
def test_blocked_split_over_field_chunks(tile):
    """n_f = 9001 > 4096: three field chunks (the last one ragged) summed in
    separate workgroups and combined in FP64; deterministic."""
    V = workloads.uniform(150, 9001, seed=61)          # dense: the accuracy case
    announce(f"2-way blocked split tile={tile}")
    c2, n2 = run2(V, acc="blocked", tile=tile)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    ea, er = check_rel(c2, ref, FP32_TOL, "c2")
    check_rel(n2, rn2, FP32_TOL, "n2")
    again, _ = run2(V, acc="blocked", tile=tile)
    assert np.array_equal(c2.view(np.uint32), again.view(np.uint32))
    plain, _ = run2(V, acc="plain", tile=tile)
    _, er_plain = check_rel(plain, ref, FP32_TOL, "c2 plain")
    print(f"dense 9001 fields: blocked max rel {er:.2e}, plain max rel {er_plain:.2e}")


def test_blocked_split_fp16():
    V32 = workloads.sparse_uniform(100, 8500, seed=62)
    V16 = workloads.to_f16(V32)
    announce("2-way blocked split fp16")
    c2, _ = run2(V16, acc="blocked")
    check_rel(c2, oracle.c2_all(V16), FP32_TOL, "c2 vs fp16 values")
    check_rel(c2, oracle.c2_all(V32), FP16_TOL, "c2 vs fp32 source")


# ------------------------------------------------------ tile shards ----

@pytest.mark.parametrize("storage,tile,acc,n_f", [("f32", 1, "plain", 333),
                                                  ("f32", 2, "auto", 5000),
                                                  ("u8", 1, "auto", 333),
                                                  ("bits", 2, "auto", 333)])
@pytest.mark.parametrize("nshards", [3, 8])
def test_shards_partition_the_pairs(storage, tile, acc, n_f, nshards):
    """ps2_compute_shard: shard k writes exactly the pairs of the upper-triangle
    tiles t = bj (bj + 1) / 2 + bi with t mod nshards == k (NaN-filled
    outputs show what was written); the shards together write every pair
    once, bit for bit as one ps2 call with the same options (with AUTO on
    5000 fields the field axis is split over chunks and the finish pass runs
    per shard); integer data equals the oracle."""
    import torch
    from paper_1705_08210_amd import ps
    n_v = 700
    if storage == "f32":
        V, kw = workloads.sparse_uniform(n_v, n_f, seed=91), {}
    elif storage == "u8":
        V, kw = workloads.levels(n_v, n_f, seed=92), dict(path="valu")
    else:
        V, kw = workloads.binary(n_v, n_f, seed=93, dtype=np.uint8), dict(path="bits", levels=1)
    Vd = to_dev(V)
    announce(f"2-way shards {storage} tile={tile} acc={acc} n_f={n_f} nshards={nshards}")
    full = host(ps.ps2(Vd, acc=acc, tile=tile, **kw)[0])
    if storage != "f32":
        check_exact_f32(full, oracle.c2_all(V), "c2")
    bm = ps.tile_configs(Vd.dtype if storage != "bits" else torch.uint8, 2)[tile - 1][0]
    i, j = np.triu_indices(n_v, 1)
    order = np.argsort(j * n_v + i, kind="stable")       # colex: (i, j) at j (j - 1) / 2 + i
    i, j = i[order], j[order]
    bi, bj = i // bm, j // bm
    owner = (bj * (bj + 1) // 2 + bi) % nshards
    m = n_v * (n_v - 1) // 2
    union = np.full(m, np.nan, dtype=np.float32)
    for k in range(nshards):
        c2 = torch.full((m,), float("nan"), device=Vd.device)
        ps.ps2_shard(Vd, k, nshards, c2=c2, acc=acc, tile=tile, **kw)
        got = host(c2)
        written = ~np.isnan(got)
        assert np.array_equal(written, owner == k), f"shard {k}"
        union[written] = got[written]
    assert np.array_equal(union.view(np.uint32), full.view(np.uint32))
