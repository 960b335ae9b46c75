"""Seeded synthetic input generators.

This module builds input matrices only.  It holds none of the similarity
arithmetic: both the HIP path and the CPU oracle consume what it produces, and
neither side imports the other.

Layout convention (used by every consumer): a matrix of ``n_v`` non-negative
vectors of ``n_f`` fields is a C-contiguous array of shape ``(n_v, n_f)``, so
the fields of one vector are contiguous.  This is the column-major storage of
the paper's ``n_f x n_v`` matrix V (Section 3.1; the input file format of
Section 6.5 is column-major as well).

All draws use numpy's PCG64 (``numpy.random.default_rng(seed)``).  Values are
drawn in float64 and cast once to the storage type (round to nearest even).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "uniform", "gwas_like", "levels", "sparse_uniform", "exponential",
    "binary", "nested_support", "to_f16", "Problem",
    "uniform_1024x256", "gwas_20000x16384", "levels_8192x32768",
    "sparse_4096x1024", "batched_64_uneven", "binary_8192x32768", "levels_4096x1024",
    "WORKLOADS",
]

_CHUNK = 1 << 22  # rows*fields generated per numpy call, bounds host memory


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _fill_rows(n_v: int, n_f: int, dtype, draw) -> np.ndarray:
    """Fill an (n_v, n_f) array chunk by chunk with ``draw(rows, n_f)``."""
    out = np.empty((n_v, n_f), dtype=dtype)
    rows = max(1, _CHUNK // max(n_f, 1))
    for r0 in range(0, n_v, rows):
        r1 = min(n_v, r0 + rows)
        out[r0:r1] = draw(r1 - r0, n_f)
    return out


def uniform(n_v: int, n_f: int, seed: int = 0, dtype=np.float32) -> np.ndarray:
    """i.i.d. U[0,1) entries."""
    g = _rng(seed)
    return _fill_rows(n_v, n_f, dtype, lambda r, f: g.random((r, f)))


def sparse_uniform(n_v: int, n_f: int, seed: int = 0, p_zero: float = 0.5,
                   dtype=np.float32) -> np.ndarray:
    """Exact zero with probability ``p_zero``, else U[0,1)."""
    g = _rng(seed)

    def draw(r, f):
        u = g.random((r, f))
        x = g.random((r, f))
        return np.where(u < p_zero, 0.0, x)
    return _fill_rows(n_v, n_f, dtype, draw)


def gwas_like(n_v: int, n_f: int, seed: int = 0, p_zero: float = 0.7,
              mean: float = 2.0, dtype=np.float32) -> np.ndarray:
    """GWAS-like strengths: exact zero w.p. ``p_zero``, else Exponential(mean)
    (a stand-in for -log10 p-value strengths of association studies)."""
    g = _rng(seed)

    def draw(r, f):
        u = g.random((r, f))
        x = g.exponential(mean, (r, f))
        return np.where(u < p_zero, 0.0, x)
    return _fill_rows(n_v, n_f, dtype, draw)


def exponential(n_v: int, n_f: int, seed: int = 0, mean: float = 1.0,
                dtype=np.float32) -> np.ndarray:
    """i.i.d. Exponential(mean) entries."""
    g = _rng(seed)
    return _fill_rows(n_v, n_f, dtype, lambda r, f: g.exponential(mean, (r, f)))


def levels(n_v: int, n_f: int, seed: int = 0,
           probs=(0.6, 0.2, 0.15, 0.05)) -> np.ndarray:
    """Integer levels 0..len(probs)-1 stored as uint8, level t drawn with
    probability ``probs[t]``."""
    g = _rng(seed)
    cum = np.cumsum(np.asarray(probs, dtype=np.float64))
    cum[-1] = 1.0

    def draw(r, f):
        u = g.random((r, f))
        return np.searchsorted(cum, u, side="right").astype(np.uint8)
    return _fill_rows(n_v, n_f, np.uint8, draw)


def binary(n_v: int, n_f: int, seed: int = 0, p_one: float = 0.3,
           dtype=np.float32) -> np.ndarray:
    """0/1 entries (the Sorensen special case), one w.p. ``p_one``."""
    g = _rng(seed)
    return _fill_rows(n_v, n_f, dtype,
                      lambda r, f: (g.random((r, f)) < p_one).astype(np.float64))


def nested_support(n_v: int, n_f: int, seed: int = 0, integer: bool = False):
    """Analytically checkable family.

    Vector i is ``a_i`` on the first ``L_i`` fields of a shared random field
    permutation ``perm`` and zero elsewhere.  ``a_i`` is dyadic in {1..8}/8
    (or an integer in {1,2,3} when ``integer``), ``L_i`` is uniform in
    [0, n_f].  Returns ``(V, a, L)`` with ``V`` float32 (uint8 when
    ``integer``); ``a`` float64, ``L`` int64.
    """
    g = _rng(seed)
    if integer:
        a = g.integers(1, 4, size=n_v).astype(np.float64)
    else:
        a = g.integers(1, 9, size=n_v).astype(np.float64) / 8.0
    L = g.integers(0, n_f + 1, size=n_v).astype(np.int64)
    perm = g.permutation(n_f)
    dt = np.uint8 if integer else np.float32
    V = np.zeros((n_v, n_f), dtype=dt)
    for i in range(n_v):
        V[i, perm[: L[i]]] = a[i]
    return V, a, L


def to_f16(V: np.ndarray) -> np.ndarray:
    """FP16 storage copy, round to nearest even."""
    return V.astype(np.float16)


# ---------------------------------------------------------------------------
# The named workloads.
# ---------------------------------------------------------------------------

def uniform_1024x256(seed: int = 0) -> np.ndarray:
    """2-way, 1024 fields x 256 vectors, FP32 U[0,1)."""
    return uniform(256, 1024, seed)


def gwas_20000x16384(seed: int = 0) -> np.ndarray:
    """2-way at scale, 20000 fields x 16384 vectors, FP32, 70% zeros,
    nonzeros Exponential(mean 2.0).  Shape of the paper's strong-scaling
    problem (Section 6.3)."""
    return gwas_like(16384, 20000, seed)


def levels_8192x32768(seed: int = 0) -> np.ndarray:
    """2-way on integer levels, 8192 fields x 32768 vectors, uint8 in
    {0,1,2,3} with probabilities 0.6/0.2/0.15/0.05."""
    return levels(32768, 8192, seed)


def sparse_4096x1024(seed: int = 0) -> np.ndarray:
    """3-way, 4096 fields x 1024 vectors, FP32 U[0,1) with 50% zeros."""
    return sparse_uniform(1024, 4096, seed, p_zero=0.5)


@dataclass
class Problem:
    n_f: int
    n_v: int
    seed: int


def batched_shapes(count: int = 64, seed: int = 0,
                   nv_range=(500, 8000), nf_range=(1000, 20000)):
    """Shapes of the uneven batch: n_v and n_f log-uniform, drawn first."""
    g = _rng(seed)
    out = []
    for p in range(count):
        n_v = int(math.floor(math.exp(g.uniform(math.log(nv_range[0]),
                                                math.log(nv_range[1])))))
        n_f = int(math.floor(math.exp(g.uniform(math.log(nf_range[0]),
                                                math.log(nf_range[1])))))
        out.append(Problem(n_f=n_f, n_v=n_v, seed=seed * 1000 + 1 + p))
    return out


def batched_64_uneven(seed: int = 0, count: int = 64, nv_range=(500, 8000),
                      nf_range=(1000, 20000)):
    """Batched uneven 2-way: ``count`` problems, n_v log-uniform in
    ``nv_range``, n_f log-uniform in ``nf_range``, FP32 Exponential(1).
    Returns a list of (n_v, n_f) float32 arrays."""
    shapes = batched_shapes(count, seed, nv_range, nf_range)
    return [exponential(p.n_v, p.n_f, p.seed) for p in shapes]


def binary_8192x32768(seed: int = 0) -> np.ndarray:
    """Binary data (the Sorensen case): 8192 fields x 32768 vectors, uint8,
    one w.p. 0.3."""
    return binary(32768, 8192, seed, p_one=0.3, dtype=np.uint8)


def levels_4096x1024(seed: int = 0) -> np.ndarray:
    """3-way on integer levels: 4096 fields x 1024 vectors, uint8 {0,1,2,3}
    with probabilities .6/.2/.15/.05 (the 3-way shape with the levels mix)."""
    return levels(1024, 4096, seed)


WORKLOADS = {
    "uniform_1024x256": uniform_1024x256,
    "gwas_20000x16384": gwas_20000x16384,
    "levels_8192x32768": levels_8192x32768,
    "sparse_4096x1024": sparse_4096x1024,
    "batched_64_uneven": batched_64_uneven,
    "binary_8192x32768": binary_8192x32768,
    "levels_4096x1024": levels_4096x1024,
}
