"""ps3_compute_noalloc, the entry point that takes its scratch from the
library's static per-GPU array, against ps3_compute with a caller workspace,
through the C ABI.  Both run the same kernels with the same tiling, so their
outputs must agree bit for bit; each is also held to the oracle.  Every case
makes two calls in a row, the second on a smaller input, so whatever the
first call left in the shared scratch must not show in the second."""

import numpy as np
import pytest

import oracle
import workloads
from psx import announce, check_exact_f32, check_rel, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _both(V, **kw):
    """(c3 from ps3_compute, c3 from ps3_compute_noalloc) on the same input."""
    import torch
    from paper_1705_08210_amd import ps
    Vd = to_dev(V)
    j_begin = kw.pop("j_begin", 1)
    j_end = kw.pop("j_end", V.shape[0] - 1)
    ref = ps.ps3(Vd, j_begin=j_begin, j_end=j_end, **kw)
    m = ps.stage_size(V.shape[0], j_begin, j_end)
    c3 = torch.full((m,), float("nan"), dtype=torch.float32, device=Vd.device)
    ps.ps3_noalloc(Vd, c3, j_begin=j_begin, j_end=j_end, **kw)
    return host(ref), host(c3)


def _same_bits(a, b, what):
    assert a.shape == b.shape, (what, a.shape, b.shape)
    bad = np.nonzero(a.view(np.uint32) != b.view(np.uint32))[0]
    assert bad.size == 0, f"{what}: {bad.size} values differ, first at {bad[0]}"


def test_fp32_sums_and_pairs_inside_then_smaller():
    for n_v, n_f, seed in [(300, 700, 71), (170, 333, 72)]:
        V = workloads.sparse_uniform(n_v, n_f, seed=seed)
        announce(f"noalloc 3-way fp32 {n_v}x{n_f}")
        ref, got = _both(V)
        _same_bits(got, ref, f"fp32 {n_v}x{n_f}")
        check_rel(got, oracle.c3_all(V), FP32_TOL, f"fp32 {n_v}x{n_f} vs oracle")


def test_fp32_blocked_split_fields_then_smaller():
    # n_f > 4096: BLOCKED field chunks, chunk partials in the scratch
    for n_v, n_f, seed in [(140, 5000, 73), (75, 4500, 74)]:
        V = workloads.gwas_like(n_v, n_f, seed=seed)
        announce(f"noalloc 3-way fp32 blocked {n_v}x{n_f}")
        ref, got = _both(V, acc="blocked")
        _same_bits(got, ref, f"blocked {n_v}x{n_f}")
        check_rel(got, oracle.c3_all(V), FP32_TOL, f"blocked {n_v}x{n_f} vs oracle")


def test_given_sums_and_pairs_stage_then_smaller():
    from paper_1705_08210_amd import ps
    import torch
    for n_v, n_f, (jb, je), seed in [(260, 900, (40, 200), 75), (120, 300, (1, 60), 76)]:
        V = workloads.sparse_uniform(n_v, n_f, seed=seed)
        announce(f"noalloc 3-way given s, n2, stage [{jb},{je}) {n_v}x{n_f}")
        Vd = to_dev(V)
        s, _ = ps.vector_sums(Vd)
        _, n2 = ps.ps2(Vd, s=s, want_c2=False, want_n2=True)
        ref = ps.ps3(Vd, s=s, n2=n2, j_begin=jb, j_end=je)
        c3 = torch.full((ps.stage_size(n_v, jb, je),), float("nan"), dtype=torch.float32,
                        device=Vd.device)
        ps.ps3_noalloc(Vd, c3, s=s, n2=n2, j_begin=jb, j_end=je)
        ref, got = host(ref), host(c3)
        _same_bits(got, ref, f"stage {n_v}x{n_f}")
        full = oracle.c3_all(V)
        lo = ps.stage_size(n_v, 1, jb)
        check_rel(got, full[lo:lo + got.size], FP32_TOL, f"stage {n_v}x{n_f} vs oracle")


@pytest.mark.parametrize("path", ["mfma", "valu"])
def test_uint8_levels_then_smaller_bit_exact(path):
    for n_v, n_f, seed in [(290, 900, 77), (133, 250, 78)]:
        V = workloads.levels(n_v, n_f, seed=seed)
        announce(f"noalloc 3-way u8 {path} {n_v}x{n_f}")
        ref, got = _both(V, path=path, levels=3)
        _same_bits(got, ref, f"u8 {path} {n_v}x{n_f}")
        check_exact_f32(got, oracle.c3_all(V), f"u8 {path} {n_v}x{n_f} vs oracle")


def test_oversized_request_is_refused_before_any_launch():
    import torch
    from paper_1705_08210_amd import ps
    n_v, n_f = 4200, 8      # the pair table alone is C(4200, 2) floats = 35 MB
    V = workloads.uniform(n_v, n_f, seed=79)
    Vd = to_dev(V)
    c3 = torch.full((ps.stage_size(n_v, 1, 2),), float("nan"), dtype=torch.float32,
                    device=Vd.device)
    announce("noalloc refusal")
    with pytest.raises(ps.PSError) as ei:
        ps.ps3_noalloc(Vd, c3, j_begin=1, j_end=2)
    assert ei.value.status == 3          # PS_ERR_WORKSPACE
    assert "static scratch" in str(ei.value)
    assert np.isnan(host(c3)).all()      # nothing written
