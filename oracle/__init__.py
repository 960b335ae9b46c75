"""CPU oracle for the Proportional Similarity metric (Section 2 of the paper).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The library under test
never imports this package, and this package imports nothing from it.

The arithmetic lives in ``ps_oracle.c`` (plain double-precision loops in
sequential field order); this module only builds and marshals.  See the C
file's header for the readings of the paper that it takes.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(hand-worked case, closed forms, library routines, brute force, invariants).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ps_oracle.c")
_LIB = os.path.join(_HERE, "libps_oracle.so")

F32, U8, F64 = 0, 2, 3


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, src]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


class Oracle:
    """ctypes view of one build of ``ps_oracle.c``."""

    def __init__(self, lib_path: str):
        lib = ctypes.CDLL(lib_path)
        P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.ps_oracle_sums.argtypes = [P, I, I64, I64, I64, P]
        lib.ps_oracle_n2.argtypes = [P, I, I64, I64, I64, I64]
        lib.ps_oracle_n2.restype = ctypes.c_double
        lib.ps_oracle_n3p.argtypes = [P, I, I64, I64, I64, I64, I64]
        lib.ps_oracle_n3p.restype = ctypes.c_double
        lib.ps_oracle_c2_all.argtypes = [P, I, I64, I64, I64, P, P]
        lib.ps_oracle_c2_pairs.argtypes = [P, I, I64, I64, P, P, P, I64, P, P]
        lib.ps_oracle_c3_all.argtypes = [P, I, I64, I64, I64, P]
        lib.ps_oracle_c3_triples.argtypes = [P, I, I64, I64, P, P, P, P, I64, P, P]
        lib.ps_oracle_set_threads.argtypes = [I]
        lib.ps_oracle_num_threads.restype = I
        self.lib = lib

    def set_threads(self, n: int) -> None:
        self.lib.ps_oracle_set_threads(int(n))

    def num_threads(self) -> int:
        return int(self.lib.ps_oracle_num_threads())

    def sums(self, V) -> np.ndarray:
        """s_i = sum_q v_{i,q}, double."""
        V, dt, n_f, n_v, ld = _prep(V)
        s = np.zeros(n_v, dtype=np.float64)
        self.lib.ps_oracle_sums(_p(V), dt, n_f, n_v, ld, _p(s))
        return s

    def n2(self, V, i: int, j: int) -> float:
        V, dt, n_f, n_v, ld = _prep(V)
        return float(self.lib.ps_oracle_n2(_p(V), dt, n_f, ld, i, j))

    def n3p(self, V, i: int, j: int, k: int) -> float:
        V, dt, n_f, n_v, ld = _prep(V)
        return float(self.lib.ps_oracle_n3p(_p(V), dt, n_f, ld, i, j, k))

    def c2_all(self, V, with_n2: bool = False):
        """All pairs i<j in colex order (index j(j-1)/2 + i)."""
        V, dt, n_f, n_v, ld = _prep(V)
        m = n_v * (n_v - 1) // 2
        c = np.zeros(m, dtype=np.float64)
        num = np.zeros(m, dtype=np.float64) if with_n2 else None
        self.lib.ps_oracle_c2_all(_p(V), dt, n_f, n_v, ld, _p(c),
                                  _p(num) if with_n2 else None)
        return (c, num) if with_n2 else c

    def c2_pairs(self, V, I, J, s=None, with_n2: bool = False):
        """Listed pairs (I[t], J[t])."""
        V, dt, n_f, n_v, ld = _prep(V)
        I = np.ascontiguousarray(I, dtype=np.int64)
        J = np.ascontiguousarray(J, dtype=np.int64)
        if s is None:
            s = self.sums(V)
        s = np.ascontiguousarray(s, dtype=np.float64)
        c = np.zeros(len(I), dtype=np.float64)
        num = np.zeros(len(I), dtype=np.float64) if with_n2 else None
        self.lib.ps_oracle_c2_pairs(_p(V), dt, n_f, ld, _p(s), _p(I), _p(J),
                                    len(I), _p(c), _p(num) if with_n2 else None)
        return (c, num) if with_n2 else c

    def c3_all(self, V) -> np.ndarray:
        """All triples i<j<k in j-slab order (j, then k, then i)."""
        V, dt, n_f, n_v, ld = _prep(V)
        m = max(n_v * (n_v - 1) * (n_v - 2) // 6, 0)
        c = np.zeros(m, dtype=np.float64)
        self.lib.ps_oracle_c3_all(_p(V), dt, n_f, n_v, ld, _p(c))
        return c

    def c3_triples(self, V, I, J, K, s=None, with_n3: bool = False):
        """Listed triples (I[t], J[t], K[t]), pairwise distinct."""
        V, dt, n_f, n_v, ld = _prep(V)
        I = np.ascontiguousarray(I, dtype=np.int64)
        J = np.ascontiguousarray(J, dtype=np.int64)
        K = np.ascontiguousarray(K, dtype=np.int64)
        if s is None:
            s = self.sums(V)
        s = np.ascontiguousarray(s, dtype=np.float64)
        c = np.zeros(len(I), dtype=np.float64)
        num = np.zeros(len(I), dtype=np.float64) if with_n3 else None
        self.lib.ps_oracle_c3_triples(_p(V), dt, n_f, ld, _p(s), _p(I), _p(J),
                                      _p(K), len(I), _p(c),
                                      _p(num) if with_n3 else None)
        return (c, num) if with_n3 else c


def _prep(V):
    """Return (array, dtype code, n_f, n_v, ld).  float16 storage is widened
    to float32 first (exact)."""
    V = np.asarray(V)
    if V.ndim != 2:
        raise ValueError("V must be (n_v, n_f)")
    if V.dtype == np.float16:
        V = V.astype(np.float32)
    if V.dtype == np.float32:
        code = F32
    elif V.dtype == np.uint8:
        code = U8
    elif V.dtype == np.float64:
        code = F64
    else:
        raise TypeError(f"unsupported dtype {V.dtype}")
    V = np.ascontiguousarray(V)
    n_v, n_f = V.shape
    return V, code, n_f, n_v, n_f


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


_default = None


def default() -> Oracle:
    """The oracle built from ``ps_oracle.c`` in this directory."""
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _default = Oracle(_LIB)
    return _default


def set_threads(n):
    default().set_threads(n)


def num_threads():
    return default().num_threads()


def sums(V):
    return default().sums(V)


def n2(V, i, j):
    return default().n2(V, i, j)


def n3p(V, i, j, k):
    return default().n3p(V, i, j, k)


def c2_all(V, with_n2=False):
    return default().c2_all(V, with_n2)


def c2_pairs(V, I, J, s=None, with_n2=False):
    return default().c2_pairs(V, I, J, s, with_n2)


def c3_all(V):
    return default().c3_all(V)


def c3_triples(V, I, J, K, s=None, with_n3=False):
    return default().c3_triples(V, I, J, K, s, with_n3)
