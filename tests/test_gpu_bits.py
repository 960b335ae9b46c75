"""BITS path (binary data, min = AND, 32 fields per word): bit-exact parity
with the CPU oracle for 2-way and 3-way, through the C ABI."""

import numpy as np
import pytest

import oracle
import workloads
from psx import (announce, check_exact_f32, host, jslab, need_gpu, sample_pairs,
                 sample_triples, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def binary_u8(n_v, n_f, seed, p_one=0.3):
    return workloads.binary(n_v, n_f, seed=seed, p_one=p_one, dtype=np.uint8)


@pytest.mark.parametrize("n_v,n_f,tile", [
    (300, 129, 0),      # 129 fields: 5 words, a 1-field tail word
    (513, 1000, 1),     # rows past a 128 tile, 32 words
    (513, 1000, 2),
    (130, 4097, 3),     # a 16-word field tile plus a 1-field tail
    (2, 1, 0),
    (65, 32, 0),        # exactly one word
    (67, 33, 0),
])
def test_bits_2way_exact(n_v, n_f, tile):
    from paper_1705_08210_amd import ps
    V = binary_u8(n_v, n_f, seed=n_v + n_f)
    announce(f"bits 2-way {n_v}x{n_f} tile={tile}")
    c2, n2 = ps.ps2(to_dev(V), path="bits", levels=1, want_n2=True, tile=tile)
    ref, rn2 = oracle.c2_all(V, with_n2=True)
    check_exact_f32(host(c2), ref, "c2")
    assert np.array_equal(host(n2).astype(np.float64), rn2)


def test_bits_match_valu_and_mfma_paths():
    """Every integer path gives the same bits on binary data."""
    from paper_1705_08210_amd import ps
    V = binary_u8(700, 2500, seed=41, p_one=0.5)
    Vd = to_dev(V)
    announce("bits vs valu vs mfma")
    outs = {p: host(ps.ps2(Vd, path=p, levels=1)[0]) for p in ("bits", "valu", "mfma",
                                                               "mfma_fp4")}
    for p in ("valu", "mfma", "mfma_fp4"):
        assert np.array_equal(outs["bits"].view(np.uint32), outs[p].view(np.uint32)), p


def test_bits_unaligned_rows():
    """Row pitch not a multiple of 16 bytes: the packing pass reads bytewise."""
    from paper_1705_08210_amd import ps
    full = binary_u8(90, 203, seed=42)
    V = full[:, :200]                       # ld = 203 bytes, n_f = 200
    import torch
    Vd = torch.from_numpy(full).cuda()[:, :200]
    announce("bits unaligned rows")
    c2, _ = ps.ps2(Vd, path="bits", levels=1)
    check_exact_f32(host(c2), oracle.c2_all(np.ascontiguousarray(V)), "c2")


@pytest.mark.parametrize("n_v,n_f,tile", [(150, 501, 0), (70, 1000, 2), (3, 1, 0),
                                          (66, 65, 0), (129, 3, 1)])
def test_bits_3way_exact(n_v, n_f, tile):
    from paper_1705_08210_amd import ps
    V = binary_u8(n_v, n_f, seed=7 * n_v + n_f, p_one=0.4)
    announce(f"bits 3-way {n_v}x{n_f} tile={tile}")
    c3 = host(ps.ps3(to_dev(V), path="bits", levels=1, tile=tile))
    check_exact_f32(c3, oracle.c3_all(V), "c3")


def test_bits_3way_stages_and_given_inputs():
    from paper_1705_08210_amd import ps
    V = binary_u8(120, 700, seed=43)
    Vd = to_dev(V)
    announce("bits 3-way stages")
    full = host(ps.ps3(Vd, path="bits", levels=1))
    parts = [host(ps.ps3(Vd, path="bits", levels=1, j_begin=a, j_end=b))
             for a, b in [(1, 2), (2, 50), (50, 119)]]
    assert np.array_equal(np.concatenate(parts).view(np.uint32), full.view(np.uint32))
    s, _ = ps.vector_sums(Vd)
    _, n2 = ps.ps2(Vd, want_c2=False, want_n2=True, path="bits", levels=1)
    given = host(ps.ps3(Vd, s=s, n2=n2, path="bits", levels=1))
    assert np.array_equal(given.view(np.uint32), full.view(np.uint32))
    # the VALU uint8 path gives the same numbers
    valu = host(ps.ps3(Vd))
    assert np.array_equal(valu.view(np.uint32), full.view(np.uint32))


def test_bits_full_size_sampled():
    """binary_8192x32768 through the bench's launch: sampled pairs exact."""
    from paper_1705_08210_amd import ps
    V = workloads.binary_8192x32768(0)
    n_v = V.shape[0]
    announce("bits 2-way 8192x32768 sampled")
    c2 = host(ps.ps2(to_dev(V), path="bits", levels=1)[0])
    i, j = sample_pairs(n_v, 4096, seed=44)
    ref = oracle.c2_pairs(V, i, j)
    check_exact_f32(c2[j * (j - 1) // 2 + i], ref, "c2 sampled")


def test_bits_3way_sampled():
    from paper_1705_08210_amd import ps
    V = binary_u8(900, 3000, seed=45)
    announce("bits 3-way 900x3000 sampled")
    c3 = host(ps.ps3(to_dev(V), path="bits", levels=1))
    i, j, k = sample_triples(900, 4096, seed=46)
    check_exact_f32(c3[jslab(900, i, j, k)], oracle.c3_triples(V, i, j, k), "c3 sampled")
