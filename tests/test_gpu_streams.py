"""Calls on a caller-given stream: the binding's workspace and outputs must
belong to that stream, so that allocations made meanwhile on the current
stream never receive their memory while the library's kernels still run."""

import numpy as np
import pytest

import oracle
import workloads
from psx import announce, check_rel, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _scribble(nbytes):
    """Allocate about nbytes on the current stream and overwrite them at once."""
    import torch
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(0xff)


def test_ps2_on_a_side_stream_with_concurrent_allocations():
    import ctypes
    import torch
    from paper_1705_08210_amd import ps
    V = workloads.gwas_like(3000, 9000, seed=71)      # BLOCKED: partials in the workspace
    Vd = to_dev(V)
    announce("2-way on a side stream")
    ref, _ = ps.ps2(Vd)
    ref = host(ref)
    o = ps._opts()
    ws_n = ps.lib.ps2_workspace_size(ps.PS_F32, V.shape[1], V.shape[0], 0, ctypes.byref(o))
    side = torch.cuda.Stream()
    for rep in range(3):
        side.wait_stream(torch.cuda.current_stream())
        c2, _ = ps.ps2(Vd, stream=side)                 # workspace freed at return
        junk = _scribble(ws_n)                          # current stream, right away
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        assert np.array_equal(host(c2).view(np.uint32), ref.view(np.uint32)), rep
        del junk
    check_rel(ref, oracle.c2_all(V), 1e-5, "c2")


def test_ps3_on_a_side_stream_with_concurrent_allocations():
    import torch
    from paper_1705_08210_amd import ps
    V = workloads.sparse_uniform(300, 5000, seed=72)   # 2 field chunks
    Vd = to_dev(V)
    announce("3-way on a side stream")
    ref = host(ps.ps3(Vd))
    side = torch.cuda.Stream()
    for rep in range(3):
        side.wait_stream(torch.cuda.current_stream())
        c3 = ps.ps3(Vd, stream=side)
        junk = _scribble(3 * ref.size * 4)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        assert np.array_equal(host(c3).view(np.uint32), ref.view(np.uint32)), rep
        del junk


def test_plan_replayed_on_another_stream():
    import torch
    from paper_1705_08210_amd import ps
    Vs = [workloads.exponential(n_v, n_f, seed=n_v) for n_v, n_f in [(300, 5000), (140, 900)]]
    Vd = [to_dev(V) for V in Vs]
    announce("batched plan on another stream")
    plan = ps.BatchedPlan(Vd)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    plan.run(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    for V, (c2, _, _) in zip(Vs, plan.outs):
        check_rel(host(c2), oracle.c2_all(V), 1e-5, f"c2 {V.shape}")
    plan.close()
