"""Pins of O2 (CPU SNN, Algorithms 1 and 2) against O1 and the mathematics.

* Exactness does not depend on the sorting direction: eq. (lower) is the
  Cauchy-Schwarz inequality and holds for any unit vector, so O2 with a
  random or adversarial direction must equal O1 bit for bit.
* The per-pair invariant |alpha_i - alpha_q| <= ||x_i - x_q|| (eq. (lower)).
* The sigma_2 = 0 special case of Section 5: for collinear data every
  candidate in the window is a neighbour.
* The decomposition of eq. (ip2) without the band (the printed algorithm)
  loses exactness under cancellation; with the band it stays exact.
"""

import numpy as np
import pytest

import oracle
from paper_2212_07679_amd import workloads as W


def same(a, b):
    return (np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
            and np.array_equal(a.dist, b.dist))


@pytest.mark.parametrize("block", [1, 64])
def test_o2_equals_o1_uniform2d(block):
    w = W.uniform2d()
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    idx = oracle.build_index(w.P)
    got, st = oracle.snn_query(idx, w.Q, w.R, block=block)
    assert same(ref, got)
    # every neighbour lies inside its query's window (sorted positions)
    pos = np.empty(idx.order.size, np.int64)
    pos[idx.order] = np.arange(idx.order.size)
    for r in range(w.m):
        p = pos[got.col[got.row_ptr[r]:got.row_ptr[r + 1]]]
        assert np.all((p >= st["lo"][r]) & (p < st["hi"][r]))


def test_o2_equals_o1_gmm16_small():
    w = W.gmm16(n=20_000, m=400, R=3.0)
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    assert ref.row_ptr[-1] > 100  # positives exercised
    idx = oracle.build_index(w.P)
    got, st = oracle.snn_query(idx, w.Q, w.R)
    assert same(ref, got)
    assert st["pairs_window"] < 0.5 * w.n * w.m  # pruning happened


@pytest.mark.parametrize("kind", ["random", "orthogonal", "axis"])
def test_o2_any_direction_is_exact(kind):
    w = W.gmm16(n=5_000, m=200, R=4.0, d=6, k=4, seed=11)
    g = np.random.default_rng(3)
    base = oracle.build_index(w.P)
    if kind == "random":
        v = g.standard_normal(w.d)
    elif kind == "orthogonal":
        v = g.standard_normal(w.d)
        v -= (v @ base.v) * base.v  # adversarial: orthogonal to v1
    else:
        v = np.zeros(w.d)
        v[-1] = 1.0
    v /= np.linalg.norm(v)
    idx = oracle.build_index(w.P, v=v)
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    got, _ = oracle.snn_query(idx, w.Q, w.R)
    assert same(ref, got)


def test_projection_lower_bound_per_pair():
    # eq. (lower): |alpha_i - alpha_q| <= ||x_i - x_q|| for every pair.
    w = W.gmm16(n=3_000, m=100, R=1.0, d=8, k=5, seed=12)
    P = w.P.astype(np.float64)
    Q = w.Q.astype(np.float64)
    idx = oracle.build_index(P)
    a_i = (P - idx.mu) @ idx.v
    a_q = (Q - idx.mu) @ idx.v
    lhs = np.abs(a_i[None, :] - a_q[:, None])
    rhs = np.sqrt(((P[None, :, :] - Q[:, None, :]) ** 2).sum(-1))
    assert np.all(lhs <= rhs * (1 + 1e-12) + 1e-12)
    assert np.isclose(np.linalg.norm(idx.v), 1.0)


def test_collinear_sigma2_zero():
    # sigma_2 = 0: all points on a line through the mean; every window
    # candidate is a neighbour (Section 5), up to the rounding widening.
    g = np.random.default_rng(5)
    u = g.standard_normal(5)
    u /= np.linalg.norm(u)
    t = g.uniform(-10, 10, 4000)
    P = 3.0 + t[:, None] * u[None, :]
    Q = P[g.choice(4000, 300, replace=False)]
    idx = oracle.build_index(P)
    sv = np.linalg.svd(P - P.mean(0), compute_uv=False)
    assert sv[1] < 1e-10 * sv[0]
    got, st = oracle.snn_query(idx, Q, 0.37, block=1)
    counts = np.diff(got.row_ptr)
    windows = st["hi"] - st["lo"]
    assert np.array_equal(counts, windows)


def test_band_needed_under_cancellation():
    # Two clusters 2e8 apart: after centring ||x|| ~ 1e8, so the decomposition
    # xbar_j - x_j.x_q loses ~u * 1e16 ~ 1 in absolute terms while R^2 = 0.01.
    g = np.random.default_rng(9)
    A = 1e8 + g.standard_normal((300, 3)) * 0.05
    B = -1e8 + g.standard_normal((300, 3)) * 0.05
    P = np.concatenate([A, B])
    Q = P[::7] + 0.01 * g.standard_normal((P[::7].shape[0], 3))
    R = 0.1
    ref = oracle.brute_radius(P, Q, R)
    idx = oracle.build_index(P)
    got, st = oracle.snn_query(idx, Q, R)
    lit, _ = oracle.snn_query(idx, Q, R, literal=True)
    assert same(ref, got)
    assert st["band"] > 0
    assert not np.array_equal(ref.col, lit.col) or not np.array_equal(ref.row_ptr, lit.row_ptr)


def test_principal_component():
    g = np.random.default_rng(2)
    X = g.standard_normal((2000, 4)) * np.array([5.0, 1.0, 0.5, 0.1])
    X -= X.mean(0)
    v = oracle.first_principal_component(X)
    w, V = np.linalg.eigh(X.T @ X)
    assert abs(abs(v @ V[:, -1]) - 1) < 1e-10
    assert v[np.argmax(np.abs(v))] > 0
    z = oracle.first_principal_component(np.zeros((10, 3)))
    assert z.tolist() == [1.0, 0.0, 0.0]
    # large-n path (eigh of X^T X) gives the same direction
    v2 = oracle.first_principal_component(X, svd_limit=0)
    assert abs(v2 @ v - 1) < 1e-10


def test_self_query_and_duplicates():
    g = np.random.default_rng(4)
    P = g.random((2000, 3))
    P[100:110] = P[5]  # exact duplicates
    idx = oracle.build_index(P)
    got, _ = oracle.snn_query(idx, P, 0.04)
    ref = oracle.brute_radius(P, P, 0.04)
    assert same(ref, got)
    row5 = got.col[got.row_ptr[5]:got.row_ptr[6]]
    assert set(range(100, 110)) <= set(row5.tolist())


def test_zero_radius():
    P = np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 0.0]])
    idx = oracle.build_index(P)
    got, _ = oracle.snn_query(idx, P, 0.0)
    assert got.col.tolist() == [0, 2, 1, 0, 2]
