"""Pins for the CPU oracle: each check ties the oracle to something other than
itself -- a hand-worked case, a library routine, a closed form, an identity,
brute force over tiny inputs, or an invariant the definitions fix.

The checks are written as functions of an oracle instance so that the
mutation test at the bottom can run them against deliberately broken builds
of the oracle source (compiled on the CPU) and show that each plausible
mistake is caught by at least one pin.
"""

import itertools
import os
import re

import numpy as np
import pytest
from scipy.spatial import distance

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers (independent of the oracle)
# ---------------------------------------------------------------------------

def read_golden(name):
    sec, out = None, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            m = re.match(r"\[(\w+)\]", line)
            if m:
                sec = m.group(1)
                out[sec] = []
                continue
            out[sec].append([float(x) for x in line.split()])
    return out


def pairs_colex(n_v):
    """Pairs (i, j), i<j, in the library's 2-way order: j major, i minor."""
    return [(i, j) for j in range(1, n_v) for i in range(j)]


def triples_jslab(n_v):
    """Triples (i, j, k), i<j<k, in the library's 3-way order: j, then k,
    then i."""
    return [(i, j, k) for j in range(1, n_v - 1) for k in range(j + 1, n_v)
            for i in range(j)]


def brute_c2(V):
    """c2 over all pairs via the absolute-difference identity
    min(a,b) = (a + b - |a-b|)/2, i.e. n2 = (s_i + s_j - sum|v_i - v_j|)/2.
    A different route to the same definition (Section 2.1)."""
    V = V.astype(np.float64)
    s = V.sum(axis=1)
    out = {}
    for i, j in itertools.combinations(range(V.shape[0]), 2):
        l1 = np.abs(V[i] - V[j]).sum()
        num = (s[i] + s[j] - l1) / 2.0
        d = s[i] + s[j]
        out[(i, j)] = 2.0 * num / d if d > 0 else 0.0
    return out


def brute_c3(V):
    """c3 over all triples via the per-field identity
    min_ij + min_ik + min_jk - min_ijk = (a + b + c) - max(a, b, c),
    so n3 = sum_q (v_i + v_j + v_k - max) (derived from Eq. 1)."""
    V = V.astype(np.float64)
    out = {}
    for i, j, k in itertools.combinations(range(V.shape[0]), 3):
        x = V[[i, j, k]]
        n3 = (x.sum(axis=0) - x.max(axis=0)).sum()
        d = x.sum()
        out[(i, j, k)] = 1.5 * n3 / d if d > 0 else 0.0
    return out


# ---------------------------------------------------------------------------
# pin checks (each asserts; each takes an oracle instance)
# ---------------------------------------------------------------------------

def check_hand_worked(orc):
    g = read_golden("hand_worked_3x3.txt")
    V = np.array(g["vectors"], dtype=np.float64)
    assert np.array_equal(orc.sums(V), np.array(g["sums"][0]))
    c2 = orc.c2_all(V)
    for (i, j, num, den), (pi, pj) in zip(g["c2"], pairs_colex(3)):
        assert (int(i), int(j)) == (pi, pj)
        assert c2[pairs_colex(3).index((pi, pj))] == num / den
    c3 = orc.c3_all(V)
    (i, j, k, num, den), = g["c3"]
    assert c3[0] == num / den
    c3t = orc.c3_triples(V, [0], [1], [2])
    assert c3t[0] == num / den


def check_braycurtis(orc):
    """c2 = 1 - BrayCurtis(u, v) for non-negative vectors, since
    sum|u-v| = s_u + s_v - 2 sum min(u, v)."""
    g = np.random.default_rng(11)
    V = g.random((9, 37)) * (g.random((9, 37)) < 0.6)
    c2 = orc.c2_all(V)
    for idx, (i, j) in enumerate(pairs_colex(9)):
        ref = 1.0 - distance.braycurtis(V[i], V[j])
        assert abs(c2[idx] - ref) <= 1e-13, (i, j)


def check_dice(orc):
    """Binary data: PS equals the Sorensen-Dice similarity (Section 2.3)."""
    V = workloads.binary(10, 50, seed=3, p_one=0.4, dtype=np.float64)
    c2 = orc.c2_all(V)
    for idx, (i, j) in enumerate(pairs_colex(10)):
        ref = 1.0 - distance.dice(V[i].astype(bool), V[j].astype(bool))
        assert abs(c2[idx] - ref) <= 1e-14, (i, j)


def check_brute_force(orc):
    """All pairs and triples of tiny integer inputs, bit-exact, in the
    library's packed orders.  n_v != n_f catches a transposed operand."""
    g = np.random.default_rng(5)
    for n_v, n_f in [(7, 13), (12, 16), (5, 1)]:
        V = g.integers(0, 5, size=(n_v, n_f)).astype(np.float32)
        V[1] = 0.0  # an all-zero vector: d may be 0
        c2 = orc.c2_all(V)
        ref2 = brute_c2(V)
        assert len(c2) == len(ref2)
        for idx, p in enumerate(pairs_colex(n_v)):
            assert c2[idx] == ref2[p], (n_v, n_f, p)
        c3 = orc.c3_all(V)
        ref3 = brute_c3(V)
        assert len(c3) == len(ref3)
        for idx, t in enumerate(triples_jslab(n_v)):
            assert c3[idx] == ref3[t], (n_v, n_f, t)
        # listed-tuple forms agree with the packed forms
        I, J = np.array(pairs_colex(n_v)).T
        assert np.array_equal(orc.c2_pairs(V, I, J), c2)
        assert np.array_equal(orc.c2_pairs(V, J, I), c2)  # symmetry
        if n_v >= 3:
            T = np.array(triples_jslab(n_v)).T
            assert np.array_equal(orc.c3_triples(V, *T), c3)
            assert np.array_equal(orc.c3_triples(V, T[2], T[0], T[1]), c3)


def check_sum_minus_max(orc):
    """n3 of Eq. 1 equals sum_q (v_i + v_j + v_k - max(v_i, v_j, v_k))."""
    V = workloads.levels(6, 40, seed=9).astype(np.float32)
    T = np.array(list(itertools.combinations(range(6), 3))).T
    _, n3 = orc.c3_triples(V, *T, with_n3=True)
    x = V.astype(np.float64)
    for t, (i, j, k) in enumerate(T.T):
        y = x[[i, j, k]]
        assert n3[t] == (y.sum(axis=0) - y.max(axis=0)).sum()


def check_scaled_copies(orc):
    """c2(u, a u) = 2 min(1,a)/(1+a); c3(u, u, a u) = 3/(2+a) for a >= 1."""
    g = np.random.default_rng(2)
    u = g.integers(0, 9, size=25).astype(np.float64)
    u[0] = 3.0
    for a in [0.25, 0.5, 1.0, 2.0, 3.0, 4.0]:
        V = np.stack([u, a * u])
        assert orc.c2_all(V)[0] == 2.0 * min(1.0, a) / (1.0 + a)
    for a in [1.0, 2.0, 4.0, 8.0]:
        V = np.stack([u, u, a * u])
        assert abs(orc.c3_all(V)[0] - 3.0 / (2.0 + a)) <= 1e-15


def check_disjoint(orc):
    """Disjoint supports: c2 = c3 = 0.  c3(u, u, w) with w disjoint from u
    equals 1.5 s_u / (2 s_u + s_w)."""
    u = np.array([1.0, 2.0, 0.0, 0.0, 4.0, 0.0])
    w = np.array([0.0, 0.0, 3.0, 5.0, 0.0, 1.0])
    x = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    assert orc.c2_all(np.stack([u, w]))[0] == 0.0
    assert orc.c3_all(np.stack([u, w, x]))[0] == 0.0
    su, sw = u.sum(), w.sum()
    assert orc.c3_all(np.stack([u, u, w]))[0] == 1.5 * su / (2 * su + sw)


def check_invariants(orc):
    """c(v,v) = 1 for s > 0; range [0,1]; vector-permutation equivariance;
    all-zero tuples give 0; scaling by 2^m leaves c unchanged."""
    g = np.random.default_rng(8)
    V = g.integers(0, 7, size=(8, 21)).astype(np.float32)
    V[3] = V[5]
    V[6] = 0.0
    c2 = orc.c2_all(V)
    pc = pairs_colex(8)
    assert c2[pc.index((3, 5))] == 1.0
    assert c2[pc.index((1, 6))] == 0.0 or V[1].sum() > 0
    assert np.all((c2 >= 0) & (c2 <= 1))
    c3 = orc.c3_all(V)
    assert np.all((c3 >= 0) & (c3 <= 1))
    Z = np.zeros((3, 4), dtype=np.float32)
    assert np.all(orc.c2_all(Z) == 0.0) and np.all(orc.c3_all(Z) == 0.0)
    perm = g.permutation(8)
    cp = orc.c2_all(V[perm])
    for idx, (i, j) in enumerate(pc):
        a, b = sorted((perm[i], perm[j]))
        assert cp[idx] == c2[pc.index((a, b))]
    tj = triples_jslab(8)
    c3p = orc.c3_all(V[perm])
    for idx, (i, j, k) in enumerate(tj):
        a, b, c = sorted((perm[i], perm[j], perm[k]))
        assert c3p[idx] == c3[tj.index((a, b, c))]
    assert np.array_equal(orc.c2_all(V * 8.0), c2)
    assert np.array_equal(orc.c3_all(V * 0.25), c3)


def check_nested_support(orc):
    """Analytic family: V[perm(q), i] = a_i [q < L_i].  Then s_i = a_i L_i,
    n2 = min(a_i,a_j) min(L_i,L_j), n3' = min(a) min(L); every value is a
    dyadic rational so the oracle must be exact."""
    V, a, L = workloads.nested_support(14, 40, seed=4)
    s = a * L
    c2 = orc.c2_all(V)
    for idx, (i, j) in enumerate(pairs_colex(14)):
        num = min(a[i], a[j]) * min(L[i], L[j])
        d = s[i] + s[j]
        assert c2[idx] == (2 * num / d if d > 0 else 0.0)
    c3 = orc.c3_all(V)
    for idx, (i, j, k) in enumerate(triples_jslab(14)):
        def n2(x, y):
            return min(a[x], a[y]) * min(L[x], L[y])
        n3 = n2(i, j) + n2(i, k) + n2(j, k) - min(a[i], a[j], a[k]) * min(L[i], L[j], L[k])
        d = s[i] + s[j] + s[k]
        assert c3[idx] == ((3 * n3) / (2 * d) if d > 0 else 0.0)


def check_sums(orc):
    V = workloads.levels(30, 77, seed=1)
    assert np.array_equal(orc.sums(V), V.astype(np.float64).sum(axis=1))
    Vf = workloads.uniform(5, 300, seed=1)
    assert np.allclose(orc.sums(Vf), Vf.astype(np.float64).sum(axis=1),
                       rtol=1e-14, atol=0)


PINS = [check_hand_worked, check_braycurtis, check_dice, check_brute_force,
        check_sum_minus_max, check_scaled_copies, check_disjoint,
        check_invariants, check_nested_support, check_sums]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_fp16_widening_is_exact(orc):
    V = workloads.to_f16(workloads.uniform(4, 64, seed=2))
    assert np.array_equal(orc.sums(V), V.astype(np.float64).sum(axis=1))


# ---------------------------------------------------------------------------
# mutation test: each plausible mistake in the oracle must fail some pin
# ---------------------------------------------------------------------------

MUTANTS = {
    # dropped n2 term in Eq. 1
    "drop_eq1_term": ("((n2ij + n2ik) + n2jk) - n3p", "(n2ij + n2ik) - n3p"),
    # wrong sign of the n3' term
    "eq1_sign": ("((n2ij + n2ik) + n2jk) - n3p", "((n2ij + n2ik) + n2jk) + n3p"),
    # missing 3/2 factor
    "c3_factor": ("(3.0 * n3) / (2.0 * d3)", "n3 / d3"),
    # missing factor 2 in c2
    "c2_factor": ("(2.0 * n2) / d2", "n2 / d2"),
    # max instead of min
    "max_not_min": ("return a < b ? a : b;", "return a > b ? a : b;"),
    # denominator uses one sum only
    "d2_one_sum": ("double d2 = si + sj;", "double d2 = si + si;"),
    # wrong operand in the 3-way term (i, i, k instead of i, j, k)
    "n3p_index": ("elem(V, dt, ld, j, q)),\n                    elem(V, dt, ld, k, q)",
                  "elem(V, dt, ld, i, q)),\n                    elem(V, dt, ld, k, q)"),
    # transposed access (q*ld + i)
    # wrong vector stride (ld - 1 instead of ld): vectors overlap
    "stride": ("int64_t at = i * ld + q;", "int64_t at = i * (ld - 1) + q;"),
    # off-by-one in the colex offset
    "colex_offset": ("int64_t idx = j * (j - 1) / 2;", "int64_t idx = (j - 1) * (j - 2) / 2;"),
    # 3-way slab loop order k/i swapped
    "slab_order": ("for (int64_t k = j + 1; k < n_v; ++k)\n            for (int64_t i = 0; i < j; ++i, ++idx) {",
                   "for (int64_t i = 0; i < j; ++i)\n            for (int64_t k = j + 1; k < n_v; ++k, ++idx) {"),
    # d = 0 convention broken (returns NaN)
    "zero_den": ("return d2 > 0.0 ? (2.0 * n2) / d2 : 0.0;", "return (2.0 * n2) / d2;"),
}


_MUTANT_RUNNER = """
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import numpy as np
import oracle
import test_oracle_pins as t
mut = oracle.Oracle({lib!r})
caught = []
for pin in t.PINS:
    try:
        with np.errstate(all="ignore"):
            pin(mut)
    except Exception:
        caught.append(pin.__name__)
print("CAUGHT", ",".join(caught))
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    """Each mutant is built and exercised in a child process, so a mutant
    that corrupts memory cannot take the test run down with it."""
    import subprocess
    import sys
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    msrc = tmp_path / "ps_oracle_mutant.c"
    msrc.write_text(src.replace(old, new, 1))
    lib = oracle.build(force=True, src=str(msrc), out=str(tmp_path / "libmut.so"))
    here = os.path.dirname(os.path.abspath(__file__))
    code = _MUTANT_RUNNER.format(root=os.path.dirname(here), tests=here, lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True,
                       text=True, timeout=300)
    if r.returncode != 0:
        # a crash (out-of-bounds access) is also a detection, but the
        # mutants are written to stay in bounds; report it
        pytest.fail(f"mutant {name} crashed the checker: {r.stderr[-400:]}")
    line = [x for x in r.stdout.splitlines() if x.startswith("CAUGHT")][-1]
    caught = [c for c in line[len("CAUGHT "):].split(",") if c]
    assert caught, f"mutant {name} passed every pin"
