"""3-way parity: the HIP path (through the C ABI) against the CPU oracle."""

import numpy as np
import pytest

import oracle
import workloads
from psx import (announce, check_exact_f32, check_rel, host, jslab, need_gpu, sample_triples,
                 to_dev)

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP16_TOL = 1e-3


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run3(V, **kw):
    from paper_1705_08210_amd import ps
    return host(ps.ps3(to_dev(V), **kw))


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_sparse_all_triples(tile):
    V = workloads.sparse_uniform(150, 501, seed=31)   # 2 tiles of 128 + tail
    announce(f"3-way sparse 150x501 tile={tile}")
    c3 = run3(V, tile=tile)
    check_rel(c3, oracle.c3_all(V), FP32_TOL, "c3")


@pytest.mark.parametrize("acc", ["plain", "blocked"])
def test_accumulation_modes(acc):
    V = workloads.gwas_like(90, 2500, seed=32)
    announce(f"3-way acc={acc}")
    check_rel(run3(V, acc=acc), oracle.c3_all(V), FP32_TOL, "c3")


@pytest.mark.parametrize("storage", ["f32", "u8"])
def test_integer_levels_bit_exact(storage):
    V = workloads.levels(140, 603, seed=33)
    if storage == "f32":
        V = V.astype(np.float32)
    announce(f"3-way integer {storage}")
    check_exact_f32(run3(V), oracle.c3_all(V), "c3")


def test_fp16_storage():
    V32 = workloads.sparse_uniform(100, 1200, seed=34)
    V16 = workloads.to_f16(V32)
    announce("3-way fp16")
    c3 = run3(V16)
    check_rel(c3, oracle.c3_all(V16), FP32_TOL, "c3 vs fp16 values")
    check_rel(c3, oracle.c3_all(V32), FP16_TOL, "c3 vs fp32 source")


@pytest.mark.parametrize("storage", ["f32", "u8"])
def test_stages_concatenate_to_full_run(storage):
    """The j-range is the restart unit of staged runs: consecutive stages,
    concatenated, equal one full run bit for bit."""
    from paper_1705_08210_amd import ps
    V = workloads.levels(120, 400, seed=35) if storage == "u8" else \
        workloads.sparse_uniform(120, 400, seed=35)
    Vd = to_dev(V)
    announce(f"3-way stages {storage}")
    full = host(ps.ps3(Vd))
    parts = [host(ps.ps3(Vd, j_begin=a, j_end=b)) for a, b in [(1, 2), (2, 40), (40, 41),
                                                                (41, 119)]]
    cat = np.concatenate(parts)
    assert cat.shape == full.shape
    assert np.array_equal(cat.view(np.uint32), full.view(np.uint32))


def test_given_sums_and_numerators_identical():
    from paper_1705_08210_amd import ps
    V = workloads.sparse_uniform(110, 700, seed=36)
    Vd = to_dev(V)
    announce("3-way given s and n2")
    s, _ = ps.vector_sums(Vd)
    _, n2 = ps.ps2(Vd, want_c2=False, want_n2=True)
    a = host(ps.ps3(Vd))
    b = host(ps.ps3(Vd, s=s, n2=n2))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("n_v,n_f", [(3, 1), (4, 2), (5, 64), (129, 3), (66, 65)])
def test_edge_sizes(n_v, n_f):
    V = workloads.sparse_uniform(n_v, n_f, seed=n_v * 7 + n_f)
    announce(f"3-way edge n_v={n_v} n_f={n_f}")
    check_rel(run3(V), oracle.c3_all(V), FP32_TOL, "c3")


def test_zero_vectors():
    V = workloads.uniform(30, 40, seed=37)
    V[[2, 3, 9]] = 0.0
    announce("3-way zero vectors")
    c3 = run3(V)
    ref = oracle.c3_all(V)
    check_rel(c3, ref, FP32_TOL, "c3")
    assert c3[jslab(30, 2, 3, 9)] == 0.0


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_nested_support_family_exact(storage):
    """n3' = min(a) min(L) on the nested-support family: every path exact."""
    n_v = 96
    V, a, L = workloads.nested_support(n_v, 1500, seed=38, integer=(storage == "u8"))
    if storage == "f16":
        V = workloads.to_f16(V)
    announce(f"3-way nested support {storage}")
    c3 = run3(V)
    j, k, i = [], [], []
    for jj in range(1, n_v - 1):
        kk, ii = np.meshgrid(np.arange(jj + 1, n_v), np.arange(jj), indexing="ij")
        j.append(np.full(kk.size, jj))
        k.append(kk.ravel())
        i.append(ii.ravel())
    i, j, k = (np.concatenate(x) for x in (i, j, k))
    idx = jslab(n_v, i, j, k)
    assert np.array_equal(idx, np.arange(len(idx)))

    def n2(x, y):
        return np.minimum(a[x], a[y]) * np.minimum(L[x], L[y])
    n3 = n2(i, j) + n2(i, k) + n2(j, k) - np.minimum(np.minimum(a[i], a[j]), a[k]) * \
        np.minimum(np.minimum(L[i], L[j]), L[k])
    d = a[i] * L[i] + a[j] * L[j] + a[k] * L[k]
    ref = np.where(d > 0, (3 * n3) / (2 * np.where(d > 0, d, 1)), 0.0)
    check_exact_f32(c3, ref, "c3")


@pytest.mark.parametrize("tile", [1, 2, 3])
def test_blocked_split_over_field_chunks(tile):
    """n_f = 8200: two field chunks for both the pair prepass and the slices."""
    from paper_1705_08210_amd import ps
    V = workloads.uniform(70, 8200, seed=39)
    announce(f"3-way blocked split tile={tile}")
    Vd = to_dev(V)
    c3 = host(ps.ps3(Vd, acc="blocked", tile=tile))
    check_rel(c3, oracle.c3_all(V), FP32_TOL, "c3")
    part = np.concatenate([host(ps.ps3(Vd, j_begin=a, j_end=b, acc="blocked", tile=tile))
                           for a, b in [(1, 30), (30, 69)]])
    assert np.array_equal(part.view(np.uint32), c3.view(np.uint32))


# ---------------------------------------------------------------------------
# 3-way on the matrix cores (uint8 levels, thermometer planes): exact.
# ---------------------------------------------------------------------------
# the int8 path's two tilings: opts.tile 0 (split: pair rows x vectors) and 2
# (whole 256-wide tiles inside each slab, 128-wide over its edges)
MFMA3 = {"mfma": dict(path="mfma"), "mfma_slab": dict(path="mfma", tile=2),
         "mfma_fp4": dict(path="mfma_fp4")}


@pytest.mark.parametrize("path", list(MFMA3))
@pytest.mark.parametrize("n_v,n_f", [(140, 603), (300, 200), (3, 1), (4, 2), (259, 5),
                                     (520, 130)])
def test_mfma_3way_exact(path, n_v, n_f):
    from paper_1705_08210_amd import ps
    V = workloads.levels(n_v, n_f, seed=n_v * 3 + n_f)
    lev = max(1, int(V.max()))
    announce(f"3-way {path} {n_v}x{n_f}")
    c3 = host(ps.ps3(to_dev(V), levels=lev, **MFMA3[path]))
    check_exact_f32(c3, oracle.c3_all(V), "c3")


@pytest.mark.parametrize("n_v,n_f,L", [(3, 64, 3), (140, 320, 3), (300, 192, 3), (520, 128, 3),
                                       (140, 320, 2), (300, 192, 1), (259, 128, 5),
                                       (200, 64, 7), (140, 128, 4), (100, 64, 6)])
def test_mfma_3way_lds_direct_stages_exact(n_v, n_f, L):
    """1..7 levels on aligned rows with n_f a multiple of 64 (the split
    tiling with its plain rows staged straight into LDS, one kernel per level
    count): every triple once (NaN-filled output), equal to the oracle and to
    the VALU path bit for bit, and stages across the split point concatenate
    to the full run."""
    import torch
    from paper_1705_08210_amd import ps
    probs = np.full(L + 1, 1.0 / (L + 1))
    V = workloads.levels(n_v, n_f, seed=n_v + n_f + L, probs=probs)
    Vd = to_dev(V)
    announce(f"3-way mfma lds-direct {n_v}x{n_f} L={L}")
    c3 = torch.full((ps.stage_size(n_v, 1, n_v - 1),), float("nan"), device=Vd.device)
    ps.ps3(Vd, c3=c3, path="mfma", levels=L)
    got = host(c3)
    assert not np.isnan(got).any()
    check_exact_f32(got, oracle.c3_all(V), "c3")
    ref = host(ps.ps3(Vd, path="valu"))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    cuts = sorted({1, max(1, n_v // 3), max(1, 2 * n_v // 3), n_v - 1})
    parts = [host(ps.ps3(Vd, j_begin=a, j_end=b, path="mfma", levels=L))
             for a, b in zip(cuts, cuts[1:])]
    assert np.array_equal(np.concatenate(parts).view(np.uint32), got.view(np.uint32))


@pytest.mark.parametrize("path", ["mfma", "mfma_fp4"])
def test_mfma_3way_stages_given_inputs_and_valu(path):
    """Stages concatenate bit for bit; given s and n2 change nothing; the
    VALU uint8 path gives the same numbers."""
    from paper_1705_08210_amd import ps
    V = workloads.levels(300, 450, seed=51)
    Vd = to_dev(V)
    announce(f"3-way {path} stages")
    full = host(ps.ps3(Vd, path=path, levels=3))
    parts = [host(ps.ps3(Vd, path=path, levels=3, j_begin=a, j_end=b))
             for a, b in [(1, 2), (2, 120), (120, 257), (257, 299)]]
    assert np.array_equal(np.concatenate(parts).view(np.uint32), full.view(np.uint32))
    s, _ = ps.vector_sums(Vd)
    _, n2 = ps.ps2(Vd, want_c2=False, want_n2=True, path=path, levels=3)
    given = host(ps.ps3(Vd, s=s, n2=n2, path=path, levels=3))
    assert np.array_equal(given.view(np.uint32), full.view(np.uint32))
    valu = host(ps.ps3(Vd, path="valu"))
    assert np.array_equal(valu.view(np.uint32), full.view(np.uint32))


@pytest.mark.parametrize("path", ["mfma", "mfma_fp4"])
def test_mfma_3way_full_size_sampled(path):
    """levels_4096x1024 in the bench's launch: sampled triples exact."""
    from paper_1705_08210_amd import ps
    from psx import sample_triples
    V = workloads.levels_4096x1024(0)
    n_v = V.shape[0]
    announce(f"3-way {path} 4096x1024 sampled")
    c3 = host(ps.ps3(to_dev(V), path=path, levels=3))
    i, j, k = sample_triples(n_v, 4096, seed=52)
    check_exact_f32(c3[jslab(n_v, i, j, k)], oracle.c3_triples(V, i, j, k), "c3 sampled")


@pytest.mark.parametrize("lo,hi,n_f", [(90, 100, 27962), (0, 100, 30000)])
def test_mfma_3way_many_levels_quotient_precision(lo, hi, n_f):
    """The fused int8 path's Eq. 1 quotient: while 6 levels n_f < 2^24 it is
    taken in FP32 from exact integer operands (the first case puts the
    denominators 2 (s_i + s_j + s_k) just under 2^24), beyond that in FP64
    (the second case).  Both must equal the oracle's FP64 quotient rounded
    once to FP32, bit for bit, and the VALU path's result."""
    from paper_1705_08210_amd import ps
    g = np.random.default_rng(n_f)
    V = g.integers(lo, hi + 1, size=(30, n_f), dtype=np.uint8)
    V[3] = 0                                   # zero denominators with zero rows
    V[4] = 0
    V[5] = 0
    announce(f"3-way mfma levels={hi} 30x{n_f}")
    Vd = to_dev(V)
    c3 = host(ps.ps3(Vd, path="mfma", levels=hi))
    check_exact_f32(c3, oracle.c3_all(V), "c3")
    valu = host(ps.ps3(Vd, path="valu"))
    assert np.array_equal(valu.view(np.uint32), c3.view(np.uint32))


def test_mfma_split_tiling_falls_back_past_32bit_offsets():
    """The split tiling of the int8 slices addresses all of V with 32-bit
    offsets (n_v ld < 2^31); a strided view past that (300 rows of stride 7.2e6
    bytes, inside the per-tile bound 256 ld < 2^31) runs the per-slab tiles
    instead, bit for bit as the VALU path and the oracle."""
    import torch
    from paper_1705_08210_amd import ps
    n_v, n_f, ld = 300, 200, 7_200_000
    V = workloads.levels(n_v, n_f, seed=57)
    big = torch.zeros((n_v, ld), dtype=torch.uint8, device="cuda")
    big[:, :n_f] = to_dev(V)
    view = big[:, :n_f]
    announce(f"3-way mfma {n_v}x{n_f} ld={ld} (slab fallback)")
    got = host(ps.ps3(view, path="mfma", levels=3))
    check_exact_f32(got, oracle.c3_all(V), "c3")
    valu = host(ps.ps3(view, path="valu"))
    assert np.array_equal(valu.view(np.uint32), got.view(np.uint32))
    del big, view
    torch.cuda.empty_cache()


# ------------------------------------------- whole tiles + edge tiles ----

def _edge_case_input(storage, n_v, n_f, seed):
    if storage == "bits":
        return workloads.binary(n_v, n_f, seed=seed, dtype=np.uint8), dict(path="bits", levels=1)
    if storage == "u8":
        return workloads.levels(n_v, n_f, seed=seed), dict(path="valu")
    V = workloads.sparse_uniform(n_v, n_f, seed=seed)
    return (workloads.to_f16(V) if storage == "f16" else V), {}


@pytest.mark.parametrize("storage", ["f32", "f16", "u8", "bits"])
@pytest.mark.parametrize("n_v", [256, 389])
def test_edge_tiles_agree_with_single_configurations(storage, n_v):
    """From n_v = 256 the library runs 128-wide tiles over the whole tiles of
    each slab rectangle and 64-wide tiles over its ragged edges (two
    launches).  Each slice sum is the same field-ordered sum in any tiling,
    so with the same pair numerators and sums the result equals a launch of
    either configuration over every tile bit for bit; a NaN-filled output
    shows that every triple is written."""
    import torch
    from paper_1705_08210_amd import ps
    V, kw = _edge_case_input(storage, n_v, 700, seed=n_v + 5)
    Vd = to_dev(V)
    announce(f"3-way edge tiles {storage} n_v={n_v}")
    s, _ = ps.vector_sums(Vd)
    _, n2 = ps.ps2(Vd, s=s, want_c2=False, want_n2=True, **kw)
    c3 = torch.full((ps.stage_size(n_v, 1, n_v - 1),), float("nan"), device=Vd.device)
    ps.ps3(Vd, s=s, n2=n2, c3=c3, **kw)
    both = host(c3)
    assert not np.isnan(both).any()
    for tile in (2, 3):      # 64-wide, 128-wide tiles over every tile of the slab
        one = host(ps.ps3(Vd, s=s, n2=n2, tile=tile, **kw))
        assert np.array_equal(both.view(np.uint32), one.view(np.uint32)), tile
    i, j, k = sample_triples(n_v, 2048, seed=n_v)
    ref = oracle.c3_triples(V, i, j, k)
    got = both[jslab(n_v, i, j, k)]
    if storage in ("u8", "bits"):
        check_exact_f32(got, ref, "c3")
    else:
        check_rel(got, ref, FP32_TOL, "c3")


def test_edge_tiles_with_field_chunks_and_stages():
    """Blocked accumulation over two field chunks and staged slabs with the
    two-launch tiling: the chunks and the stages combine exactly as in a
    single-configuration launch."""
    from paper_1705_08210_amd import ps
    n_v = 300
    V = workloads.gwas_like(n_v, 5000, seed=91)
    Vd = to_dev(V)
    announce("3-way edge tiles, blocked chunks and stages")
    s, _ = ps.vector_sums(Vd)
    _, n2 = ps.ps2(Vd, s=s, acc="blocked", want_c2=False, want_n2=True)
    full = host(ps.ps3(Vd, s=s, n2=n2, acc="blocked"))
    one = host(ps.ps3(Vd, s=s, n2=n2, acc="blocked", tile=3))
    assert np.array_equal(full.view(np.uint32), one.view(np.uint32))
    cuts = [1, 2, 130, 131, 257, n_v - 1]
    parts = [host(ps.ps3(Vd, s=s, n2=n2, acc="blocked", j_begin=a, j_end=b))
             for a, b in zip(cuts, cuts[1:])]
    assert np.array_equal(np.concatenate(parts).view(np.uint32), full.view(np.uint32))
    i, j, k = sample_triples(n_v, 1024, seed=92)
    check_rel(full[jslab(n_v, i, j, k)], oracle.c3_triples(V, i, j, k), FP32_TOL, "c3")


@pytest.mark.parametrize("path", list(MFMA3))
@pytest.mark.parametrize("n_v", [300, 600])
def test_mfma_whole_and_edge_tiles(path, n_v):
    """Every tiling of the matrix-core slices writes each triple once
    (NaN-filled output) and equals the VALU result bit for bit; stages
    concatenate to the full run.  The split tiling's two parts meet at
    j = 2 n_v / 5 (120 and 240 here), inside the stages below; the slab
    tiling runs whole 256-wide tiles (from n_v = 513 there are some) and
    128-wide tiles over the rest."""
    import torch
    from paper_1705_08210_amd import ps
    V = workloads.levels(n_v, 333, seed=n_v + 7)
    Vd = to_dev(V)
    announce(f"3-way {path} tilings n_v={n_v}")
    c3 = torch.full((ps.stage_size(n_v, 1, n_v - 1),), float("nan"), device=Vd.device)
    ps.ps3(Vd, c3=c3, levels=3, **MFMA3[path])
    got = host(c3)
    assert not np.isnan(got).any()
    ref = host(ps.ps3(Vd, path="valu"))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    cuts = [1, 200, 257, n_v - 1]
    parts = [host(ps.ps3(Vd, j_begin=a, j_end=b, levels=3, **MFMA3[path]))
             for a, b in zip(cuts, cuts[1:])]
    assert np.array_equal(np.concatenate(parts).view(np.uint32), got.view(np.uint32))
    i, j, k = sample_triples(n_v, 2048, seed=n_v + 8)
    check_exact_f32(got[jslab(n_v, i, j, k)], oracle.c3_triples(V, i, j, k), "c3")


@pytest.mark.parametrize("kind", ["f32", "u8_mfma", "f32_stage_given"])
def test_3way_plan_replays_match_eager(kind):
    """A 3-way stage captured into a HIP graph (ps_plan_create_3way) replays
    the eager result bit for bit, three times, with other eager work and
    synchronisations between the replays."""
    import torch
    from paper_1705_08210_amd import ps
    n_v = 300
    if kind == "u8_mfma":
        V = workloads.levels(n_v, 1500, seed=82)
        kw = dict(path="mfma", levels=3)
    else:
        V = workloads.sparse_uniform(n_v, 1500, seed=81)
        kw = {}
    Vd = to_dev(V)
    jb, je = (50, 220) if kind == "f32_stage_given" else (1, n_v - 1)
    s = n2 = None
    if kind == "f32_stage_given":
        s, _ = ps.vector_sums(Vd)
        _, n2 = ps.ps2(Vd, s=s, want_c2=False, want_n2=True)
    announce(f"3-way plan {kind}")
    eager = host(ps.ps3(Vd, s=s, n2=n2, j_begin=jb, j_end=je, **kw))
    plan = ps.Plan3(Vd, s=s, n2=n2, j_begin=jb, j_end=je, **kw)
    for rep in range(3):
        plan.c3.fill_(float("nan"))
        ps.ps2(Vd)                     # other eager work between replays
        torch.cuda.synchronize()
        got = host(plan.run())
        assert np.array_equal(got.view(np.uint32), eager.view(np.uint32)), rep
    plan.close()
    lo = ps.stage_size(n_v, 1, jb)
    ref = oracle.c3_all(V)[lo:lo + eager.size]
    if kind == "u8_mfma":
        check_exact_f32(eager, ref, "c3")
    else:
        check_rel(eager, ref, FP32_TOL, "c3")
