"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times: sampled outputs against the oracle one by
one, and the nested-support family checked in full against its closed form."""

import math

import numpy as np
import pytest

import oracle
import workloads
from psx import (announce, check_exact_f32, check_rel, colex, host, jslab, need_gpu,
                 sample_pairs, sample_triples, to_dev)

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP16_TOL = 1e-3
NSAMPLE = 1 << 14


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_gwas_20000x16384_sampled():
    from paper_1705_08210_amd import ps
    V = workloads.gwas_20000x16384()
    announce("scale 2-way gwas 20000x16384 f32 (bench configuration)")
    Vd = to_dev(V)
    s, bad = ps.vector_sums(Vd)
    c2, _ = ps.ps2(Vd, s=s)
    c2 = host(c2)
    assert host(bad)[0] == 0
    assert np.all((c2 >= 0) & (c2 <= 1 + 1e-6))
    I, J = sample_pairs(V.shape[0], NSAMPLE, seed=3)
    ea, er = check_rel(c2[colex(I, J)], oracle.c2_pairs(V, I, J), FP32_TOL, "c2")
    print(f"gwas sampled max abs {ea:.3e} max rel {er:.3e}")
    # equal vectors give exactly-1 (N2 in FP32, s in FP64): within tolerance
    assert c2.shape[0] == V.shape[0] * (V.shape[0] - 1) // 2


@pytest.mark.parametrize("path", ["valu", "mfma", "mfma_fp4"])
def test_levels_8192x32768_sampled_exact(path):
    from paper_1705_08210_amd import ps
    V = workloads.levels_8192x32768()
    announce(f"scale 2-way levels 8192x32768 u8 path={path}")
    c2, n2 = ps.ps2(to_dev(V), want_n2=True, path=path, levels=3)
    c2, n2 = host(c2), host(n2)
    I, J = sample_pairs(V.shape[0], NSAMPLE, seed=4)
    ref, rn2 = oracle.c2_pairs(V, I, J, with_n2=True)
    check_exact_f32(c2[colex(I, J)], ref, "c2")
    assert np.array_equal(n2[colex(I, J)].astype(np.float64), rn2)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_sparse_4096x1024_3way_sampled(storage):
    from paper_1705_08210_amd import ps
    V32 = workloads.sparse_4096x1024()
    V = workloads.to_f16(V32) if storage == "f16" else V32
    announce(f"scale 3-way sparse 4096x1024 {storage}")
    c3 = host(ps.ps3(to_dev(V)))
    assert c3.shape[0] == math.comb(1024, 3)
    I, J, K = sample_triples(1024, NSAMPLE, seed=5)
    got = c3[jslab(1024, I, J, K)]
    check_rel(got, oracle.c3_triples(V, I, J, K), FP32_TOL, "c3 vs storage values")
    if storage == "f16":
        ea, er = check_rel(got, oracle.c3_triples(V32, I, J, K), FP16_TOL, "c3 vs fp32 source")
        print(f"fp16 storage vs fp32 source: max abs {ea:.3e} max rel {er:.3e}")


@pytest.mark.parametrize("kind", ["f32", "u8_mfma", "u8_mfma_lds"])
def test_nested_support_2way_full_size_exact(kind):
    """Every one of the 1.34e8 outputs at the benchmark's size, against the
    closed form, bit for bit: FP32 data on the VALU tiles, integer levels on
    the int8 matrix-core half tiles (n_f = 20000 with register staging; a
    multiple of 64 fields with staging straight into LDS)."""
    from paper_1705_08210_amd import ps
    n_v, n_f = 16384, 19968 if kind == "u8_mfma_lds" else 20000
    V, a, L = workloads.nested_support(n_v, n_f, seed=51, integer=kind != "f32")
    announce(f"scale 2-way nested support {n_f}x{n_v} {kind} full")
    kw = dict(path="mfma", levels=3) if kind.startswith("u8_mfma") else {}
    c2 = host(ps.ps2(to_dev(V), **kw)[0])
    del V
    s = a * L
    for j0 in range(1, n_v, 1024):
        j1 = min(n_v, j0 + 1024)
        jj = np.repeat(np.arange(j0, j1), np.arange(j0, j1))
        ii = np.concatenate([np.arange(j) for j in range(j0, j1)])
        num = np.minimum(a[ii], a[jj]) * np.minimum(L[ii], L[jj])
        d = s[ii] + s[jj]
        ref = np.where(d > 0, 2 * num / np.where(d > 0, d, 1), 0.0)
        check_exact_f32(c2[colex(ii, jj)], ref, f"c2 columns {j0}..{j1}")


@pytest.mark.parametrize("kind", ["f32", "u8_mfma", "u8_valu"])
def test_nested_support_3way_full_size_exact(kind):
    """Every one of the 1.78e8 triples of the 3-way benchmark's shape against
    the closed form, bit for bit: FP32 data on the VALU slices, integer levels
    on the int8 matrix-core split tiling (the bench's integer 3-way launch)
    and on the uint8 VALU slices."""
    from paper_1705_08210_amd import ps
    n_v, n_f = 1024, 4096
    V, a, L = workloads.nested_support(n_v, n_f, seed=52, integer=kind != "f32")
    announce(f"scale 3-way nested support 4096x1024 {kind} full")
    kw = {"f32": {}, "u8_mfma": dict(path="mfma", levels=3),
          "u8_valu": dict(path="valu")}[kind]
    c3 = host(ps.ps3(to_dev(V), **kw))
    s = a * L
    pos = 0
    for j in range(1, n_v - 1):
        kk, ii = np.meshgrid(np.arange(j + 1, n_v), np.arange(j), indexing="ij")
        kk, ii = kk.ravel(), ii.ravel()

        def n2(x, y):
            return np.minimum(a[x], a[y]) * np.minimum(L[x], L[y])
        n3 = n2(ii, j) + n2(ii, kk) + n2(j, kk) - np.minimum(np.minimum(a[ii], a[j]), a[kk]) * \
            np.minimum(np.minimum(L[ii], L[j]), L[kk])
        d = s[ii] + s[j] + s[kk]
        ref = np.where(d > 0, (3 * n3) / (2 * np.where(d > 0, d, 1)), 0.0)
        check_exact_f32(c3[pos:pos + len(ref)], ref, f"c3 slab {j}")
        pos += len(ref)
    assert pos == c3.shape[0]


def test_sparse_4096x1024_3way_full_oracle():
    """The 3-way bench workload compared in full: every one of the C(1024, 3)
    triples against the oracle (about half a minute of oracle time on 16
    host threads)."""
    from paper_1705_08210_amd import ps
    V = workloads.sparse_4096x1024()
    announce("scale 3-way sparse 4096x1024 f32, all triples against the oracle")
    c3 = host(ps.ps3(to_dev(V)))
    ea, er = check_rel(c3, oracle.c3_all(V), FP32_TOL, "c3")
    print(f"3-way full: max abs {ea:.3e} max rel {er:.3e} over {c3.size} triples")


@pytest.mark.parametrize("path", ["mfma", "mfma_fp4", "valu"])
def test_levels_3way_full_oracle_exact(path):
    """Integer 3-way in full (600 vectors x 4096 fields, several 256-wide
    tiles per slab): every triple bit-exact against the oracle."""
    from paper_1705_08210_amd import ps
    V = workloads.levels(600, 4096, seed=53)
    announce(f"scale 3-way levels 4096x600 {path}, all triples against the oracle")
    c3 = host(ps.ps3(to_dev(V), path=path, levels=3))
    check_exact_f32(c3, oracle.c3_all(V), "c3")
