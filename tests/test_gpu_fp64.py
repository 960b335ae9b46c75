"""FP64 data (the paper's double-precision build): FP64 min and accumulation,
FP64 numerators, c2/c3 rounded once to FP32.  Parity with the FP64 oracle:
the only error left is the final FP32 rounding (relative 2^-24) plus the
summation-order difference of FP64 sums (~1e-16 n_f relative)."""

import numpy as np
import pytest

import oracle
import workloads
from psx import (announce, check_exact_f32, check_rel, host, jslab, need_gpu, sample_triples,
                 to_dev)

pytestmark = pytest.mark.gpu

OUT_TOL = 6.5e-8      # one rounding to FP32 (2^-24 = 5.96e-8) plus FP64 order effects
N2_TOL = 1e-12


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("n_v,n_f,tile", [(300, 1000, 0), (130, 777, 1), (130, 777, 2),
                                          (130, 777, 3), (2, 1, 0), (67, 3, 0)])
def test_fp64_2way(n_v, n_f, tile):
    from paper_1705_08210_amd import ps
    V = workloads.sparse_uniform(n_v, n_f, seed=n_v + n_f, dtype=np.float64)
    announce(f"fp64 2-way {n_v}x{n_f} tile={tile}")
    c2, n2 = ps.ps2(to_dev(V), want_n2=True, tile=tile)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_rel(host(c2), ref, OUT_TOL, "c2")
    assert n2.dtype.is_floating_point and n2.element_size() == 8
    check_rel(host(n2), rn2, N2_TOL, "n2")


def test_fp64_integer_values_exact():
    """Integer-valued FP64 data: every sum is exact, so c2 is bit-exact."""
    from paper_1705_08210_amd import ps
    V = workloads.levels(200, 1500, seed=71).astype(np.float64)
    announce("fp64 integer values")
    c2, n2 = ps.ps2(to_dev(V), want_n2=True)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_exact_f32(host(c2), ref, "c2")
    assert np.array_equal(host(n2), rn2)


def test_fp64_unaligned_rows_and_sums():
    """Row pitch of an odd number of doubles (element-wise staging), and the
    FP64 sums with their out-of-domain count."""
    import torch
    from paper_1705_08210_amd import ps
    big = workloads.gwas_like(90, 511, seed=72, dtype=np.float64)
    V = np.ascontiguousarray(big[:, :500])
    Vd = torch.from_numpy(big).cuda()[:, :500]
    announce("fp64 unaligned rows")
    c2, _ = ps.ps2(Vd)
    check_rel(host(c2), oracle.c2_all(V), OUT_TOL, "c2")
    s, bad = ps.vector_sums(Vd)
    check_rel(host(s), oracle.sums(V), 1e-13, "s")
    assert host(bad)[0] == 0
    W = big.copy()
    W[3, 7], W[5, 9], W[6, 10] = -1.0, np.inf, np.nan
    _, bad = ps.vector_sums(torch.from_numpy(W).cuda())
    assert host(bad)[0] == 3


@pytest.mark.parametrize("n_v,n_f,tile", [(150, 501, 0), (70, 1200, 3), (3, 1, 0)])
def test_fp64_3way(n_v, n_f, tile):
    from paper_1705_08210_amd import ps
    V = workloads.sparse_uniform(n_v, n_f, seed=7 * n_v + n_f, dtype=np.float64)
    announce(f"fp64 3-way {n_v}x{n_f} tile={tile}")
    c3 = host(ps.ps3(to_dev(V), tile=tile))
    check_rel(c3, oracle.c3_all(V), OUT_TOL, "c3")


def test_fp64_3way_stages_and_given_inputs():
    from paper_1705_08210_amd import ps
    V = workloads.exponential(120, 800, seed=73, dtype=np.float64)
    Vd = to_dev(V)
    announce("fp64 3-way stages")
    full = host(ps.ps3(Vd))
    parts = [host(ps.ps3(Vd, j_begin=a, j_end=b)) for a, b in [(1, 2), (2, 60), (60, 119)]]
    assert np.array_equal(np.concatenate(parts).view(np.uint32), full.view(np.uint32))
    s, _ = ps.vector_sums(Vd)
    _, n2 = ps.ps2(Vd, want_c2=False, want_n2=True)
    given = host(ps.ps3(Vd, s=s, n2=n2))
    assert np.array_equal(given.view(np.uint32), full.view(np.uint32))


def test_fp64_3way_sampled_large():
    from paper_1705_08210_amd import ps
    V = workloads.sparse_uniform(700, 3000, seed=74, dtype=np.float64)
    announce("fp64 3-way 700x3000 sampled")
    c3 = host(ps.ps3(to_dev(V)))
    i, j, k = sample_triples(700, 4096, seed=75)
    check_rel(c3[jslab(700, i, j, k)], oracle.c3_triples(V, i, j, k), OUT_TOL, "c3")


def test_fp64_batched_is_unsupported():
    from paper_1705_08210_amd import ps
    Vs = [to_dev(workloads.uniform(20, 30, seed=76, dtype=np.float64))]
    with pytest.raises(ps.PSError) as e:
        ps.ps2_batched(Vs)
    assert e.value.status == 5
