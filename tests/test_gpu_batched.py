"""Batched 2-way: many uneven problems in one launch (and as a
captured plan) against one launch per problem and against the oracle."""

import numpy as np
import pytest

import oracle
import workloads
from psx import announce, check_exact_f32, check_rel, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def small_batch(seed=0, count=12, integer=False):
    g = np.random.default_rng(seed)
    out = []
    for p in range(count):
        n_v = int(g.integers(2, 700))
        n_f = int(g.integers(1, 3000))
        if integer:
            out.append(workloads.levels(n_v, n_f, seed=100 + p))
        else:
            out.append(workloads.exponential(n_v, n_f, seed=100 + p))
    return out


@pytest.mark.parametrize("tile", [1, 2])
def test_batched_matches_per_problem_and_oracle(tile):
    from paper_1705_08210_amd import ps
    Vs = small_batch(1)
    announce(f"batched 12 problems tile={tile}")
    Vd = [to_dev(V) for V in Vs]
    # same accumulation on both sides (with acc=auto a small single problem
    # may be split over field chunks for parallelism, which the batch is not)
    outs = ps.ps2_batched(Vd, tile=tile, want_n2=True, acc="plain")
    for V, Vx, (c2, n2, _) in zip(Vs, Vd, outs):
        a, an2 = ps.ps2(Vx, tile=tile, want_n2=True, acc="plain")
        assert np.array_equal(host(c2).view(np.uint32), host(a).view(np.uint32))
        assert np.array_equal(host(n2).view(np.uint32), host(an2).view(np.uint32))
        check_rel(host(c2), oracle.c2_all(V), 1e-5, f"c2 {V.shape}")


def test_batched_integer_exact():
    from paper_1705_08210_amd import ps
    Vs = small_batch(2, count=9, integer=True)
    announce("batched u8")
    outs = ps.ps2_batched([to_dev(V) for V in Vs])
    for V, (c2, _, _) in zip(Vs, outs):
        check_exact_f32(host(c2), oracle.c2_all(V), f"c2 {V.shape}")


def test_plan_replays_match_eager():
    """The captured plan is replayed several times with other eager work in
    between; every replay must equal the eager batched result."""
    import torch
    from paper_1705_08210_amd import ps
    Vs = small_batch(3, count=10)
    Vd = [to_dev(V) for V in Vs]
    announce("batched plan replays")
    eager = [host(c) for c, _, _ in ps.ps2_batched(Vd, tile=1)]
    plan = ps.BatchedPlan(Vd, tile=1)
    for rep in range(4):
        for c, _, _ in plan.outs:
            c.fill_(-1.0)
        _ = torch.rand(1000, device="cuda").sum()        # unrelated eager work
        ps.ps2(Vd[0], tile=2)
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for e, (c, _, _) in zip(eager, plan.outs):
            assert np.array_equal(e.view(np.uint32), host(c).view(np.uint32)), rep
    plan.close()


def test_batched_with_given_sums_and_edge_problems():
    from paper_1705_08210_amd import ps
    import torch
    Vs = [workloads.exponential(n_v, n_f, seed=n_v) for n_v, n_f in
          [(1, 10), (2, 1), (300, 5), (129, 513)]]
    Vd = [to_dev(V) for V in Vs]
    announce("batched edge problems")
    outs = []
    for V in Vd:
        s, _ = ps.vector_sums(V)
        m = V.shape[0] * (V.shape[0] - 1) // 2
        outs.append((torch.empty(m, device="cuda"), None, s))
    ps.ps2_batched(Vd, outs=outs)
    for V, (c2, _, _) in zip(Vs, outs):
        check_rel(host(c2), oracle.c2_all(V), 1e-5, f"c2 {V.shape}")


def test_mixed_dtypes_rejected():
    from paper_1705_08210_amd import ps
    with pytest.raises(TypeError):
        ps.ps2_batched([to_dev(workloads.uniform(5, 5)), to_dev(workloads.levels(5, 5))])
