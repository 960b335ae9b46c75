"""Shared helpers of the GPU tests (no similarity arithmetic here beyond the
packed index formulas of the output layouts)."""

import sys

import numpy as np
import pytest


def announce(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a dying run shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(V: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(V)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def colex(i, j):
    """2-way packed index of pair (i, j), i < j."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return j * (j - 1) // 2 + i


def slab_off(n, j):
    j = np.asarray(j, dtype=np.int64)
    return (n - 1) * (j * (j - 1) // 2) - ((j - 1) * j * (2 * j - 1)) // 6


def jslab(n, i, j, k, j_begin=1):
    """3-way packed index of triple (i, j, k), i < j < k, relative to the
    first triple of slab j_begin."""
    i, j, k = (np.asarray(x, dtype=np.int64) for x in (i, j, k))
    return slab_off(n, j) - slab_off(n, j_begin) + (k - j - 1) * j + i


def sample_pairs(n_v, m, seed):
    g = np.random.default_rng(seed)
    a = g.integers(0, n_v, size=m)
    b = g.integers(0, n_v - 1, size=m)
    b = np.where(b >= a, b + 1, b)
    return np.minimum(a, b), np.maximum(a, b)


def sample_triples(n_v, m, seed):
    g = np.random.default_rng(seed)
    out = []
    while sum(len(x) for x in out) < m:
        t = np.sort(g.integers(0, n_v, size=(m, 3)), axis=1)
        ok = (t[:, 0] < t[:, 1]) & (t[:, 1] < t[:, 2])
        out.append(t[ok])
    t = np.concatenate(out)[:m]
    return t[:, 0], t[:, 1], t[:, 2]


def check_rel(gpu, ref, tol, what=""):
    """|gpu - ref| <= tol * ref where ref > 0, and gpu == 0 exactly where
    ref == 0.  Returns (max abs err, max rel err)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    assert np.all(np.isfinite(gpu)), f"{what}: non-finite output"
    zero = ref == 0
    assert np.all(gpu[zero] == 0), f"{what}: nonzero where the reference is 0"
    err = np.abs(gpu - ref)
    rel = np.where(zero, 0.0, err / np.where(zero, 1.0, np.abs(ref)))
    worst = int(np.argmax(rel)) if rel.size else 0
    assert rel.size == 0 or rel.max() <= tol, (
        f"{what}: max rel err {rel.max():.3e} > {tol:g} at {worst} "
        f"(gpu {gpu[worst]!r}, ref {ref[worst]!r})")
    return (float(err.max()) if err.size else 0.0, float(rel.max()) if rel.size else 0.0)


def check_exact_f32(gpu, ref64, what=""):
    """Bit-exact: the GPU float32 equals the float64 reference rounded once."""
    gpu = np.asarray(gpu)
    ref32 = np.asarray(ref64, dtype=np.float64).astype(np.float32)
    bad = np.nonzero(gpu.view(np.uint32) != ref32.view(np.uint32))[0]
    assert bad.size == 0, (f"{what}: {bad.size} mismatches, first at {bad[0]}: "
                           f"gpu {gpu[bad[0]]!r} ref {ref64[bad[0]]!r}")
