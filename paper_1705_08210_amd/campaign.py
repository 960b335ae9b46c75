"""Staged 3-way campaigns (the staging of Section 4.2 and the output handling
of Section 6.5).

The triples are computed one stage (a range of middle indices j) at a time
into a device buffer, reduced on the device (one byte per metric, or a
thresholded (index, value) list), copied to pinned host memory on a second
stream and handed to a caller-supplied sink -- while the next two stages are
already queued, so the sink's host work overlaps GPU work.  Consecutive
stages alternate between two compute streams, so one stage's last
workgroups run beside the next stage's first ones instead of leaving the
GPU partly idle at every stage boundary.  Three buffer sets rotate; a device
buffer is reused only after its copy has completed, a host buffer only after
the sink has returned.  The per-vector sums and pair numerators are computed
once and stay resident.

    from paper_1705_08210_amd import campaign
    campaign.run3(V, n_stages=8, sink=lambda st: ..., reduce="u8")

Every step runs in libps through the C ABI (ps.py); this module only orders
the calls on two streams.
"""

from __future__ import annotations

import atexit
import dataclasses
import math

import torch

from . import ps


def release() -> None:
    """Free the pinned host blocks that campaigns leave in torch's host-memory
    cache (their staging buffers), with the HIP runtime fully up.  Registered
    to run at interpreter exit, so no page-locked block is left for the
    runtime's own teardown (exit-time destructors run after tools that
    intercept HIP calls, such as a profiler, may have shut down); call it
    earlier to return the memory sooner."""
    if not torch.cuda.is_initialized():
        return
    torch.cuda.synchronize()
    empty = getattr(torch._C, "_host_emptyCache", None)
    if empty is not None:
        empty()


atexit.register(release)


def stage_bounds(n_v: int, n_stages: int) -> list[tuple[int, int]]:
    """Split the middle indices [1, n_v - 1) into at most n_stages consecutive
    ranges with about equal numbers of triples (slab j holds j (n_v - 1 - j)).
    Every range is non-empty; together they cover [1, n_v - 1)."""
    if n_v < 3:
        return []
    n_stages = max(1, min(int(n_stages), n_v - 2))
    total = ps.stage_size(n_v, 1, n_v - 1)
    bounds, j = [], 1
    for k in range(1, n_stages + 1):
        if j >= n_v - 1:
            break
        if k == n_stages:
            bounds.append((j, n_v - 1))
            break
        target = total * k / n_stages
        e = j + 1
        while e < n_v - 1 and ps.stage_size(n_v, 1, e) < target:
            e += 1
        bounds.append((j, e))
        j = e
    return bounds


@dataclasses.dataclass
class Stage:
    """One finished stage as the sink receives it (host memory, valid only
    during the call; copy what must be kept)."""
    index: int
    j_begin: int
    j_end: int
    first: int                    # packed j-slab index of the stage's first triple
    size: int                     # triples in the stage
    u8: torch.Tensor | None = None        # reduce="u8": one byte per triple
    c3: torch.Tensor | None = None        # reduce="none": float32 per triple
    idx: torch.Tensor | None = None       # reduce="threshold": global packed indices
    val: torch.Tensor | None = None       #   and their values
    dropped: int = 0              # threshold entries beyond the capacity


def run3(V: torch.Tensor, n_stages: int, sink, reduce: str = "u8", threshold: float = 0.0,
         cap: int | None = None, path: str = "auto", levels: int = 0, acc: str = "auto",
         tile: int = 0) -> int:
    """Compute all triples of V stage by stage; returns the number of stages.

    reduce: "u8" (one byte per metric), "threshold" (entries >= threshold,
    at most `cap` per stage, default the stage size) or "none" (float32).
    The sink is called in stage order from this thread."""
    if reduce not in ("u8", "threshold", "none"):
        raise ValueError(f"unknown reduce {reduce!r}")
    n_v = V.shape[0]
    stages = stage_bounds(n_v, n_stages)
    if not stages:
        return 0
    dev = V.device
    main = torch.cuda.current_stream(dev)
    computes = [torch.cuda.Stream(dev) for _ in range(2)]   # default priority
    copy = torch.cuda.Stream(dev)
    s, _ = ps.vector_sums(V, want_bad=False)
    _, n2 = ps.ps2(V, s=s, want_c2=False, want_n2=True, path=path, levels=levels, acc=acc,
                   tile=tile)
    ready = torch.cuda.Event()
    ready.record(main)
    for cs in computes:
        cs.wait_event(ready)
    biggest = max(ps.stage_size(n_v, a, b) for a, b in stages)
    cap_ = biggest if cap is None else int(cap)
    nbuf = min(3, len(stages))      # stage k uses buffer set k % nbuf
    c3 = [torch.empty(biggest, dtype=torch.float32, device=dev) for _ in range(nbuf)]
    if reduce == "u8":
        dout = [torch.empty(biggest, dtype=torch.uint8, device=dev) for _ in range(nbuf)]
        hout = [torch.empty(biggest, dtype=torch.uint8, pin_memory=True) for _ in range(nbuf)]
    elif reduce == "none":
        dout = c3
        hout = [torch.empty(biggest, dtype=torch.float32, pin_memory=True) for _ in range(nbuf)]
    else:
        hidx = [torch.empty(max(cap_, 1), dtype=torch.int64, pin_memory=True)
                for _ in range(nbuf)]
        hval = [torch.empty(max(cap_, 1), dtype=torch.float32, pin_memory=True)
                for _ in range(nbuf)]
        hcnt = [torch.empty(1, dtype=torch.int64, pin_memory=True) for _ in range(nbuf)]
        dsel = [None] * nbuf
    copied = [None] * nbuf    # event: the buffer set's copy to the host has finished

    def launch(k):
        """Compute, reduce and start the copy of stage k on buffer set k % nbuf
        (its previous stage has been delivered: the host buffer is free)."""
        b = k % nbuf
        a, e = stages[k]
        m = ps.stage_size(n_v, a, e)
        compute = computes[k % 2]
        with torch.cuda.stream(compute):
            if copied[b] is not None:             # the buffer's previous copy is done
                compute.wait_event(copied[b])
            out = c3[b][:m]
            ps.ps3(V, s=s, n2=n2, j_begin=a, j_end=e, c3=out, acc=acc, tile=tile, path=path,
                   levels=levels)
            if reduce == "u8":
                ps.quantize_u8(out, out=dout[b][:m])
            elif reduce == "threshold":
                dsel[b] = ps.threshold(out, threshold, base=ps.stage_size(n_v, 1, a), cap=cap_)
            done = torch.cuda.Event()
            done.record(compute)
        copy.wait_event(done)
        with torch.cuda.stream(copy):
            if reduce == "threshold":
                idx, val, cnt = dsel[b]
                hidx[b][:cap_].copy_(idx[:cap_], non_blocking=True)
                hval[b][:cap_].copy_(val[:cap_], non_blocking=True)
                hcnt[b].copy_(cnt, non_blocking=True)
            else:
                hout[b][:m].copy_(dout[b][:m], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(copy)
        copied[b] = ev

    def deliver(k):
        b = k % nbuf
        a, e = stages[k]
        m = ps.stage_size(n_v, a, e)
        copied[b].synchronize()
        st = Stage(index=k, j_begin=a, j_end=e, first=ps.stage_size(n_v, 1, a), size=m)
        if reduce == "u8":
            st.u8 = hout[b][:m]
        elif reduce == "none":
            st.c3 = hout[b][:m]
        else:
            cnt = int(hcnt[b][0])
            kept = min(cnt, cap_)
            st.idx, st.val, st.dropped = hidx[b][:kept], hval[b][:kept], cnt - kept
        sink(st)

    ahead = nbuf - 1            # stages queued while the oldest one is delivered
    for k in range(ahead):
        launch(k)
    for k in range(len(stages)):
        if k + ahead < len(stages):
            launch(k + ahead)   # its set was used by stage k - 1, delivered already
        deliver(k)
    copy.synchronize()          # every stage's copy, hence every stage, has finished
    for cs in computes:
        cs.synchronize()
    main.wait_stream(copy)
    # nothing of this call outlives it: events, device and pinned buffers go
    # back to torch's caches now (release() frees the pinned ones)
    copied.clear()
    del c3
    if reduce == "threshold":
        del hidx, hval, hcnt, dsel
    else:
        del dout, hout
    return len(stages)


def expected_bytes(n_v: int) -> int:
    """Size of a full u8 campaign output: one byte per triple."""
    return math.comb(n_v, 3)
