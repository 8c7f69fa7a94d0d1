"""Pins of O1 (normative brute force) against exact arithmetic and lattice counts.

None of these re-types the oracle's formula: the references are exact
rational arithmetic, integer lattice counts computed with integer square
roots, IEEE identities and the direct-form error bound gamma_{d+2} proved in
Section 4.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2212_07679_amd import workloads as W

U64 = 2.0**-53


def gamma(k):
    return k * U64 / (1 - k * U64)


def lattice_count(r2: int, centre, lo: int, hi: int, d: int) -> int:
    """Integer points z in [lo, hi]^d with ||z - centre||^2 <= r2, counted
    with integer arithmetic only (centre integral)."""
    def rec(k, rem):
        if k == d:
            return 1
        c = centre[k]
        tot = 0
        t = math.isqrt(rem)
        for x in range(max(lo, c - t), min(hi, c + t) + 1):
            dx2 = (x - c) ** 2
            if dx2 <= rem:
                tot += rec(k + 1, rem - dx2)
        return tot
    return rec(0, r2)


def test_gauss_circle_inclusive():
    # N(5) = 81 integer points with x^2 + y^2 <= 25; 12 of them lie exactly on
    # the circle, so a strict comparison would return 69.
    P = W.lattice(-6, 6, 2)
    nb = oracle.brute_radius(P, np.zeros((1, 2)), 5.0)
    assert nb.row_ptr[-1] == 81 == lattice_count(25, (0, 0), -6, 6, 2)
    on_circle = np.isclose(nb.dist, 5.0)
    assert on_circle.sum() == 12


@pytest.mark.parametrize("centre,r2,lo,hi,d", [
    ((3, 4), 25, -3, 10, 2),      # off-centre query in an asymmetric range: sign of p - q
    ((2, -1, 5), 9, -4, 8, 3),     # 3-D
    ((8, 0), 25, -3, 10, 2),       # clipped by the range: each centre coordinate matters
    ((7, -3, 0), 9, -4, 8, 3),
    ((1, 2, 3, 0, 1), 4, -2, 4, 5),
    ((0, 0, 0), 10, -4, 4, 3),       # r^2 not a square: R = fl(sqrt(10)) and fl(R*R) rounds
])
def test_lattice_offcentre(centre, r2, lo, hi, d):
    P = W.lattice(lo, hi, d)
    q = np.array(centre, dtype=np.float64)[None, :]
    R = math.sqrt(r2)
    nb = oracle.brute_radius(P, q, R)
    # Integer squared distances are computed exactly by the normative sum, so
    # the count is that of integer points with ||z - c||^2 <= fl(R*R), i.e.
    # <= r2 when fl(R*R) >= r2 and <= r2 - 1 otherwise.
    expect = lattice_count(r2 if R * R >= r2 else r2 - 1, centre, lo, hi, d)
    assert nb.row_ptr[-1] == expect
    ids = nb.col
    diff = P[ids] - q
    assert np.all(np.sum(diff * diff, axis=1) <= r2)


def _rand_cases():
    g = np.random.default_rng(12345)
    for d in (1, 2, 3, 5, 8):
        for kind in ("f64", "f32", "far"):
            n, m = 60, 8
            P = g.standard_normal((n, d))
            if kind == "f32":
                P = P.astype(np.float32).astype(np.float64)
            if kind == "far":
                P = 1e6 + P * 1e-3
            Q = np.concatenate([P[:3], P[g.integers(0, n, 5)] + 1e-4 * g.standard_normal((5, d))])
            yield d, kind, P, Q


@pytest.mark.parametrize("d,kind,P,Q", list(_rand_cases()))
def test_o1_vs_exact(d, kind, P, Q):
    """|S - S*| <= gamma_{d+2} S* for every pair (Section 4's direct-form bound),
    and O1's set equals the exact set except for pairs inside that bound of R^2."""
    Sx = [[oracle.exact_sqdist(p, q) for p in P] for q in Q]
    # radius: the median exact distance of the first query, so sets are non-trivial,
    # plus a radius equal to an attained distance (a tie in exact arithmetic).
    s_sorted = sorted(float(s) for s in Sx[0])
    for R in (math.sqrt(s_sorted[len(s_sorted) // 2]), math.sqrt(s_sorted[5])):
        nb = oracle.brute_radius(P, Q, R)
        sets_exact, _ = oracle.exact_radius(P, Q, R)
        R2 = R * R
        R2x = Fraction(R) ** 2
        for r, q in enumerate(Q):
            S = oracle.normative_sqdist(P, q)
            for i in range(P.shape[0]):
                err = abs(Fraction(float(S[i])) - Sx[r][i])
                assert err <= Fraction(gamma(d + 2)) * Sx[r][i]
            got = set(nb.col[nb.row_ptr[r]:nb.row_ptr[r + 1]].tolist())
            exact = set(sets_exact[r])
            for i in got ^ exact:
                slack = Fraction(gamma(d + 2)) * Sx[r][i] + abs(Fraction(R2) - R2x)
                assert abs(Sx[r][i] - R2x) <= slack, (r, i)
            # ids ascending, distances = fl32(sqrt(S)) within 1e-6 of the exact value
            row = nb.col[nb.row_ptr[r]:nb.row_ptr[r + 1]]
            assert np.all(np.diff(row) > 0)
            for i, dd in zip(row.tolist(), nb.dist[nb.row_ptr[r]:nb.row_ptr[r + 1]].tolist()):
                ex = math.sqrt(float(Sx[r][i]))
                assert abs(dd - ex) <= 1e-6 * max(ex, 1e-300)


def test_self_inclusion_and_symmetry():
    w = W.uniform2d(n=500, m=500, R=0.1, seed=7)
    P = w.P
    nb = oracle.brute_radius(P, P, w.R)
    n = P.shape[0]
    for i in range(n):
        row = nb.col[nb.row_ptr[i]:nb.row_ptr[i + 1]]
        k = np.searchsorted(row, i)
        assert row[k] == i and nb.dist[nb.row_ptr[i] + k] == 0.0
    # IEEE: fl(a - b) = -fl(b - a), so S(p_i, p_j) == S(p_j, p_i) bitwise and
    # the neighbour relation of a self-query is symmetric.
    pairs = set()
    for i in range(n):
        for j in nb.col[nb.row_ptr[i]:nb.row_ptr[i + 1]].tolist():
            pairs.add((i, j))
    assert all((j, i) in pairs for (i, j) in pairs)


def test_zero_radius_and_duplicates():
    P = np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 0.0], [1.0, 1.0 + 2**-52]])
    nb = oracle.brute_radius(P, P[:2], 0.0)
    assert nb.col.tolist() == [0, 2, 1]


def test_empty_inputs():
    P = np.zeros((5, 3))
    nb = oracle.brute_radius(P, np.zeros((0, 3)), 1.0)
    assert nb.row_ptr.tolist() == [0] and nb.col.size == 0
    with pytest.raises(ValueError):
        oracle.brute_radius(P, np.zeros((1, 3)), -1.0)
    with pytest.raises(ValueError):
        oracle.brute_radius(P, np.zeros((1, 3)), float("nan"))


def test_no_fma_in_normative_sum():
    # t = (2^-27, 2^-27, 1 + 2^-30).  Left to right the partial sum is
    # 2^-53 exactly; fl(t_2^2) = 1 + 2^-29 (the 2^-60 term is rounded off), and
    # 2^-53 + 1 + 2^-29 is a tie that rounds to even: S = 1 + 2^-29.  A fused
    # multiply-add keeps the 2^-60 term, breaks the tie upwards and gives
    # 1 + 2^-29 + 2^-52.
    p = np.array([[2.0**-27, 2.0**-27, 1.0 + 2.0**-30]])
    s = oracle.normative_sqdist(p, np.zeros(3))[0]
    assert s == 1.0 + 2.0**-29


def test_left_to_right_order():
    # t = (1, 2^-27, 2^-27, 2^-27): adding 2^-54 to 1 three times left to right
    # leaves 1; summing the small terms first (pairwise or reversed) gives
    # 3 * 2^-54 = 0.75 ulp(1) and rounds to 1 + 2^-52.
    p = np.array([[1.0, 2.0**-27, 2.0**-27, 2.0**-27]])
    s = oracle.normative_sqdist(p, np.zeros(4))[0]
    assert s == 1.0
