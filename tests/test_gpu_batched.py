"""Batched 2-way: many uneven problems in one launch (and as a
captured plan) against one launch per problem and against the oracle."""

import numpy as np
import pytest

import oracle
import workloads
from psx import (announce, check_exact_f32, check_rel, colex, host, need_gpu, sample_pairs,
                 to_dev)

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


# ------------------------------------------- field-chunk split in a batch ----

# (n_v, n_f): more than 4096 fields split into 4096-field chunks under AUTO
# and BLOCKED, with ragged last chunks (9001 = 2 x 4096 + 809, 4097 = 4096 + 1),
# whole chunks only (12288), exactly one chunk (4096, not split), unsplit
# problems, a one-pair problem with two chunks and a problem without pairs.
CHUNK_SHAPES = [(257, 9001), (130, 4096), (200, 4097), (64, 12288), (311, 2000),
                (2, 5000), (1, 7000), (145, 8192 + 130)]


def chunk_batch(seed=11):
    return [workloads.exponential(n_v, n_f, seed=seed + t)
            for t, (n_v, n_f) in enumerate(CHUNK_SHAPES)]


@pytest.mark.parametrize("acc", ["auto", "blocked"])
@pytest.mark.parametrize("tile", [0, 2])
def test_batched_field_chunks_match_oracle(acc, tile):
    """Split and unsplit problems in one launch: every c2 and n2 against the
    oracle, and bit-identical to a single-problem launch with the same
    field-chunk split (blocked: the same chunks summed in the same order)."""
    from paper_1705_08210_amd import ps
    Vs = chunk_batch()
    Vd = [to_dev(V) for V in Vs]
    announce(f"batched field chunks acc={acc} tile={tile}")
    outs = ps.ps2_batched(Vd, acc=acc, tile=tile, want_n2=True)
    worst = 0.0
    for V, Vx, (c2, n2, _) in zip(Vs, Vd, outs):
        if V.shape[0] < 2:
            assert c2.numel() == 0
            continue
        ref, rn2 = oracle.c2_all(V, with_n2=True)
        _, er = check_rel(host(c2), ref, 1e-5, f"c2 {V.shape}")
        check_rel(host(n2), rn2, 1e-5, f"n2 {V.shape}")
        worst = max(worst, er)
        if tile:
            one, one_n2 = ps.ps2(Vx, acc="blocked", tile=tile, want_n2=True)
            assert np.array_equal(host(c2).view(np.uint32), host(one).view(np.uint32)), V.shape
            assert np.array_equal(host(n2).view(np.uint32), host(one_n2).view(np.uint32))
    print(f"batched field chunks acc={acc} tile={tile}: max rel err {worst:.2e}")


@pytest.mark.parametrize("acc", ["auto", "blocked"])
def test_batched_field_chunks_plan_equals_eager(acc):
    """The captured plan of a split batch replays the eager result bit for
    bit, with other work on the stream between replays."""
    import torch
    from paper_1705_08210_amd import ps
    Vs = chunk_batch(seed=21)
    Vd = [to_dev(V) for V in Vs]
    announce(f"batched field chunks plan acc={acc}")
    eager = [host(c) for c, _, _ in ps.ps2_batched(Vd, acc=acc)]
    plan = ps.BatchedPlan(Vd, acc=acc)
    for rep in range(3):
        for c, _, _ in plan.outs:
            c.fill_(float("nan"))
        ps.ps2(Vd[0], acc="plain")                     # unrelated work in between
        torch.cuda.synchronize()
        plan.run()
        for e, (c, _, _) in zip(eager, plan.outs):
            assert np.array_equal(e.view(np.uint32), host(c).view(np.uint32)), rep
    plan.close()
    for V, e in zip(Vs, eager):
        if V.shape[0] >= 2:
            check_rel(e, oracle.c2_all(V), 1e-5, f"c2 {V.shape}")


def test_batched_call_returns_before_the_work_is_done():
    """The batched call enqueues its table writes as kernels and does not
    wait on the host: with the stream held busy by an earlier call, it
    returns while that work is still running, and the results are right."""
    import time
    import torch
    from paper_1705_08210_amd import ps
    big = to_dev(workloads.exponential(4096, 8192, seed=5))      # ~2.3 ms per call
    Vs = chunk_batch(seed=31)
    Vd = [to_dev(V) for V in Vs]
    outs = ps._batch_outputs(Vd)
    announce("batched call without a host wait")
    ps.ps2(big, acc="plain")                          # warm-up (workspace, kernels)
    ps.ps2_batched(Vd, outs=outs)
    torch.cuda.synchronize()
    busy = torch.cuda.Event()
    for _ in range(8):                                # ~18 ms of queued work
        ps.ps2(big, acc="plain")
    busy.record()
    t0 = time.perf_counter()
    ps.ps2_batched(Vd, outs=outs)
    dt = time.perf_counter() - t0
    still_busy = not busy.query()
    torch.cuda.synchronize()
    assert still_busy, "the earlier work finished before the batched call returned"
    print(f"batched call returned after {dt * 1e3:.2f} ms")
    for V, (c2, _, _) in zip(Vs, outs):
        if V.shape[0] >= 2:
            check_rel(host(c2), oracle.c2_all(V), 1e-5, f"c2 {V.shape}")


def test_batched_64_uneven_full_size_sampled():
    """The benchmark's batch (64 problems, 35 of them split over field
    chunks) as the benchmark runs it, a captured plan with library choices:
    sampled pairs of every problem against the oracle."""
    from paper_1705_08210_amd import ps
    Vs = workloads.batched_64_uneven(0)
    announce("batched_64_uneven full size, plan, 256 pairs per problem")
    Vd = [to_dev(V) for V in Vs]
    plan = ps.BatchedPlan(Vd)
    plan.run()
    worst = 0.0
    split = 0
    for p, (V, (c2, _, _)) in enumerate(zip(Vs, plan.outs)):
        c2 = host(c2)
        I, J = sample_pairs(V.shape[0], 256, seed=1000 + p)
        _, er = check_rel(c2[colex(I, J)], oracle.c2_pairs(V, I, J), 1e-5, f"problem {p}")
        worst = max(worst, er)
        split += V.shape[1] > 4096
    plan.close()
    assert split == 35
    print(f"batched_64_uneven: 64 problems x 256 pairs, max rel err {worst:.2e}")
