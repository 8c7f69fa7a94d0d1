"""Pins of the Section 2 distances in the oracle (oracle/metrics.py), CPU only.

* Manhattan: exact rational 1-norms on random inputs (every disagreement
  with the float64 rule within its rounding bound), integer-lattice counts of
  the 1-ball by enumeration (ties at the boundary included), the 1-norm ball
  inside the 2-norm ball;
* normalisation: exactly representable cases, norms within the rounding
  bound, scale invariance by powers of two;
* angular and cosine: unit vectors at known angles on a circle, and random
  directions against angles from arccos away from the boundary.
"""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.metrics import (angular_threshold, brute_angular, brute_cosine, brute_l1, cosine_threshold, manhattan,
                            normalize_rows, snn_angular)
from paper_2212_07679_amd import workloads as W

U64 = 2.0**-53


def gamma(k):
    return k * U64 / (1 - k * U64)


def test_manhattan_against_exact_rationals():
    g = np.random.default_rng([2212, 7679, 91])
    for d in (1, 3, 7, 16):
        P = g.standard_normal((200, d)) * 10.0 ** g.integers(-3, 3, size=(200, 1))
        q = g.standard_normal(d)
        m = manhattan(P, q)
        for i in range(P.shape[0]):
            exact = sum(abs(Fraction(float(P[i, k])) - Fraction(float(q[k]))) for k in range(d))
            assert abs(Fraction(float(m[i])) - exact) <= Fraction(gamma(d + 1)) * exact
        R = float(np.median(m))
        nb = brute_l1(P, q, R)
        exact_set = {i for i in range(P.shape[0])
                     if sum(abs(Fraction(float(P[i, k])) - Fraction(float(q[k]))) for k in range(d)) <= Fraction(R)}
        got = set(nb.col.tolist())
        # any disagreement lies inside the rounding band of M
        for i in got ^ exact_set:
            assert abs(m[i] - R) <= gamma(d + 1) * R * 2


def lattice_l1_count(r, centre, lo, hi, d):
    return sum(1 for x in itertools.product(range(lo, hi + 1), repeat=d)
               if sum(abs(a - c) for a, c in zip(x, centre)) <= r)


@pytest.mark.parametrize("d,r,centre,lo,hi", [(2, 3, (0, 0), -5, 5), (2, 4, (3, -1), -4, 6), (3, 3, (1, 1, 1), -3, 4),
                                              (4, 2, (0, 0, 0, 0), -3, 3)])
def test_manhattan_lattice_counts(d, r, centre, lo, hi):
    P = W.lattice(lo, hi, d)
    nb = brute_l1(P, np.array([centre], dtype=np.float64), float(r))
    assert nb.row_ptr[-1] == lattice_l1_count(r, centre, lo, hi, d)
    # the boundary is inclusive and the query itself is a neighbour
    below = brute_l1(P, np.array([centre], dtype=np.float64), float(np.nextafter(r, 0)))
    assert nb.row_ptr[-1] > below.row_ptr[-1]


def test_manhattan_ball_inside_euclidean_ball():
    g = np.random.default_rng([2212, 7679, 92])
    P = g.random((2000, 5))
    Q = g.random((20, 5))
    l1 = brute_l1(P, Q, 0.4)
    l2 = oracle.brute_radius(P, Q, 0.4)
    for j in range(Q.shape[0]):
        a = set(l1.col[l1.row_ptr[j]:l1.row_ptr[j + 1]].tolist())
        b = set(l2.col[l2.row_ptr[j]:l2.row_ptr[j + 1]].tolist())
        assert a <= b and len(a) < len(b)


def test_normalize_exact_cases():
    X = np.array([[3.0, 4.0], [1.0, 1.0], [0.0, -2.0**40], [2.0**-500, 0.0]])
    Y = normalize_rows(X)
    assert Y[0, 0] == float(Fraction(3, 5)) and Y[0, 1] == float(Fraction(4, 5))
    assert Y[2, 1] == -1.0 and Y[2, 0] == 0.0 and Y[3, 0] == 1.0
    # 1/sqrt(2), correctly rounded through the float64 quotient
    assert Y[1, 0] == Y[1, 1] == 1.0 / math.sqrt(2.0)
    X4 = np.ones((1, 4))
    assert np.all(normalize_rows(X4) == 0.5)
    with pytest.raises(ValueError):
        normalize_rows(np.zeros((1, 3)))
    with pytest.raises(ValueError):
        normalize_rows(np.array([[1.0, np.nan]]))
    with pytest.raises(ValueError):  # the squared sum underflows to zero
        normalize_rows(np.array([[1e-300, 0.0]]))


def test_normalize_norms_and_scaling():
    g = np.random.default_rng([2212, 7679, 93])
    for d in (1, 2, 17, 100):
        X = g.standard_normal((300, d))
        Y = normalize_rows(X)
        n2 = np.array([sum(Fraction(float(v)) ** 2 for v in row) for row in Y[:30]])
        assert all(abs(float(x) - 1.0) <= 4 * gamma(d + 2) for x in n2)
        assert np.array_equal(normalize_rows(X * 2.0**37), Y)  # power-of-two scaling is exact
        Y32 = normalize_rows(X.astype(np.float32))
        assert Y32.dtype == np.float32


def test_angular_on_a_circle():
    step = math.radians(7.0)
    ang = np.arange(40) * step
    X = np.stack([np.cos(ang), np.sin(ang)], axis=1) * 3.0  # not unit length before normalising
    Y = normalize_rows(X)
    nb = brute_angular(Y, Y, math.radians(20.0))
    for k in range(40):
        want = [j for j in range(40) if abs(j - k) <= 2]  # 14 degrees in, 21 out
        got = nb.col[nb.row_ptr[k]:nb.row_ptr[k + 1]]
        assert got.tolist() == want
        # reported distances are the angles themselves
        ref = np.radians(7.0 * np.abs(np.array(want) - k))
        assert np.allclose(nb.dist[nb.row_ptr[k]:nb.row_ptr[k + 1]], ref, rtol=1e-5, atol=1e-6)
    # cosine distance 1 - cos(14 deg) lies between the 2- and 3-step neighbours
    c = 1.0 - math.cos(math.radians(17.0))
    nbc = brute_cosine(Y, Y, c)
    for k in range(40):
        want = [j for j in range(40) if abs(j - k) <= 2]
        assert nbc.col[nbc.row_ptr[k]:nbc.row_ptr[k + 1]].tolist() == want
        ref = 1.0 - np.cos(np.radians(7.0 * np.abs(np.array(want) - k)))
        assert np.allclose(nbc.dist[nbc.row_ptr[k]:nbc.row_ptr[k + 1]], ref, rtol=1e-5, atol=1e-7)


def test_angular_thresholds():
    # the squared chord of an angle: 60 degrees on unit vectors is a chord of 1
    assert abs(angular_threshold(math.pi / 3) - 1.0) <= 4 * U64
    assert angular_threshold(0.0) == 0.0 and angular_threshold(math.pi) == 4.0
    assert cosine_threshold(0.25) == 0.5
    for bad in (-0.1, math.pi + 1e-9, float("nan")):
        with pytest.raises(ValueError):
            angular_threshold(bad)
    with pytest.raises(ValueError):
        cosine_threshold(-1.0)


def test_angular_and_cosine_random_directions():
    g = np.random.default_rng([2212, 7679, 94])
    X = g.standard_normal((600, 8))
    Y = normalize_rows(X)
    alpha = 1.0
    nb = brute_angular(Y, Y[:40], alpha)
    cosines = np.clip(Y[:40] @ Y.T, -1.0, 1.0)
    theta = np.arccos(cosines)
    for j in range(40):
        far = np.abs(theta[j] - alpha) > 1e-9
        want = np.flatnonzero((theta[j] <= alpha) & far)
        got = nb.col[nb.row_ptr[j]:nb.row_ptr[j + 1]]
        assert set(want.tolist()) == set(got.tolist()) & set(np.flatnonzero(far).tolist())
        assert np.allclose(nb.dist[nb.row_ptr[j]:nb.row_ptr[j + 1]], theta[j][got], rtol=1e-5, atol=1e-6)
    c = 0.3
    nbc = brute_cosine(Y, Y[:40], c)
    for j in range(40):
        far = np.abs((1.0 - cosines[j]) - c) > 1e-9
        want = np.flatnonzero((1.0 - cosines[j] <= c) & far)
        got = nbc.col[nbc.row_ptr[j]:nbc.row_ptr[j + 1]]
        assert set(want.tolist()) == set(got.tolist()) & set(np.flatnonzero(far).tolist())
        assert np.allclose(nbc.dist[nbc.row_ptr[j]:nbc.row_ptr[j + 1]], 1.0 - cosines[j][got], rtol=1e-5,
                           atol=1e-7)
    # the CPU SNN with the squared chord gives the same sets (eq. (lower) on unit rows)
    idx = oracle.build_index(Y)
    nbs, _ = snn_angular(idx, Y[:40], alpha)
    assert np.array_equal(nbs.row_ptr, nb.row_ptr) and np.array_equal(nbs.col, nb.col)
    assert np.allclose(nbs.dist, nb.dist, rtol=1e-5)


def _lattice_pins_hold():
    for d, r, centre, lo, hi in [(2, 3, (0, 0), -5, 5), (2, 4, (3, -1), -4, 6), (3, 3, (1, 1, 1), -3, 4)]:
        P = W.lattice(lo, hi, d)
        nb = brute_l1(P, np.array([centre], dtype=np.float64), float(r))
        if nb.row_ptr[-1] != lattice_l1_count(r, centre, lo, hi, d):
            return False
    return True


@pytest.mark.parametrize("kind", ["squared", "drop_last", "plus", "max"])
def test_lattice_pins_catch_planted_mistakes(monkeypatch, kind):
    import oracle.metrics as M

    def wrong(P, q):
        P = np.asarray(P, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64).reshape(-1)
        ks = range(P.shape[1] - 1) if kind == "drop_last" else range(P.shape[1])
        s = np.zeros(P.shape[0])
        for k in ks:
            t = P[:, k] + q[k] if kind == "plus" else P[:, k] - q[k]
            s = np.maximum(s, np.abs(t)) if kind == "max" else s + (t * t if kind == "squared" else np.abs(t))
        return s

    assert _lattice_pins_hold()
    monkeypatch.setattr(M, "manhattan", wrong)
    assert not _lattice_pins_hold()
