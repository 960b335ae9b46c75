"""Staged 3-way campaigns and the on-device output reduction."""

import numpy as np
import pytest

import oracle
import workloads
from psx import announce, check_rel, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_quantize_u8_definition():
    """One byte per metric: rint(255 * clamp(c, 0, 1)), ties to even,
    including the tails of a length that is not a multiple of 4."""
    import torch
    from paper_1705_08210_amd import ps
    g = np.random.default_rng(61)
    c = g.random(10_003).astype(np.float32)
    c[:8] = [0.0, 1.0, -0.5, 2.0, 0.5 / 255, 1.5 / 255, 127.5 / 255, 254.5 / 255]
    announce("quantize u8")
    q = host(ps.quantize_u8(torch.from_numpy(c).cuda()))
    want = np.rint(np.clip(c, 0, 1) * np.float32(255)).astype(np.uint8)
    assert np.array_equal(q, want)
    off = host(ps.quantize_u8(torch.from_numpy(c).cuda()[1:]))   # unaligned start
    assert np.array_equal(off, want[1:])


@pytest.mark.parametrize("n,thr,cap", [(100_000, 0.9, None), (5_000, 0.0, None),
                                       (70_001, 0.99, 50), (3, 2.0, None), (0, 0.5, None)])
def test_threshold_selects_in_index_order(n, thr, cap):
    import torch
    from paper_1705_08210_amd import ps
    g = np.random.default_rng(62)
    c = g.random(n).astype(np.float32)
    announce(f"threshold n={n} thr={thr} cap={cap}")
    idx, val, cnt = ps.threshold(torch.from_numpy(c).cuda(), thr, base=7, cap=cap)
    cnt = int(host(cnt)[0])
    sel = np.nonzero(c >= np.float32(thr))[0]
    assert cnt == sel.size
    kept = sel.size if cap is None else min(cap, sel.size)
    assert np.array_equal(host(idx)[:kept], sel[:kept] + 7)
    assert np.array_equal(host(val)[:kept], c[sel[:kept]])


@pytest.mark.parametrize("reduce", ["u8", "none", "threshold"])
def test_campaign_stages_equal_one_full_run(reduce):
    from paper_1705_08210_amd import campaign, ps
    V = workloads.sparse_uniform(200, 900, seed=63)
    Vd = to_dev(V)
    announce(f"campaign reduce={reduce}")
    full = ps.ps3(Vd)
    got = []
    n = campaign.run3(Vd, n_stages=5, sink=lambda st: got.append(
        (st.first, st.size, None if st.u8 is None else st.u8.clone(),
         None if st.c3 is None else st.c3.clone(),
         None if st.idx is None else (st.idx.clone(), st.val.clone(), st.dropped))),
        reduce=reduce, threshold=0.6)
    assert n == 5 and [g[0] for g in got] == sorted(g[0] for g in got)
    assert sum(g[1] for g in got) == full.numel()
    fullh = host(full)
    if reduce == "u8":
        cat = np.concatenate([g[2].numpy() for g in got])
        assert np.array_equal(cat, host(ps.quantize_u8(full)))
    elif reduce == "none":
        cat = np.concatenate([g[3].numpy() for g in got])
        assert np.array_equal(cat.view(np.uint32), fullh.view(np.uint32))
        check_rel(cat, oracle.c3_all(V), 1e-5, "campaign c3")
    else:
        idx = np.concatenate([g[4][0].numpy() for g in got])
        val = np.concatenate([g[4][1].numpy() for g in got])
        assert all(g[4][2] == 0 for g in got)
        sel = np.nonzero(fullh >= np.float32(0.6))[0]
        assert np.array_equal(idx, sel)
        assert np.array_equal(val, fullh[sel])


def test_campaign_integer_bytes_match_oracle():
    """Integer data through the MFMA path: each byte equals the rounded
    oracle value (c3 is exact, so the byte is unique)."""
    from paper_1705_08210_amd import campaign
    V = workloads.levels(180, 700, seed=64)
    announce("campaign integer u8")
    parts = []
    campaign.run3(to_dev(V), n_stages=3, sink=lambda st: parts.append(st.u8.clone()),
                  reduce="u8", path="mfma", levels=3)
    ref = oracle.c3_all(V).astype(np.float32)
    want = np.rint(np.clip(ref, 0, 1) * np.float32(255)).astype(np.uint8)
    assert np.array_equal(np.concatenate([p.numpy() for p in parts]), want)
