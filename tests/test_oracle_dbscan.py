"""Pins of the DBSCAN oracle (oracle/dbscan.py), CPU only.

* scikit-learn's DBSCAN -- the implementation Section 6.4 runs with SNN as
  its radius search -- on seeded clustered data (labels must agree exactly;
  the data are checked to hold no pair whose squared distance is within a
  relative 1e-9 of eps^2, where two correct distance evaluations could
  disagree);
* closed-form configurations: isolated points, a unit-spaced line at the
  inclusive boundary, a border point shared by two clusters (lowest-numbered
  cluster wins, in both index orders), min_samples = 1 (components).
"""

import numpy as np
import pytest

import oracle
from oracle.dbscan import dbscan, dbscan_from_neighbors

sklearn_cluster = pytest.importorskip("sklearn.cluster")


def blobs(seed, n, d, k, std, noise_frac):
    g = np.random.default_rng([2212, 7679, 90, seed])
    centres = g.uniform(0.0, 1.0, size=(k, d))
    nb = int(round(n * (1 - noise_frac)))
    lab = g.integers(0, k, size=nb)
    P = np.concatenate([centres[lab] + std * g.standard_normal((nb, d)), g.uniform(0.0, 1.0, size=(n - nb, d))])
    return P[g.permutation(n)]


def no_boundary_pairs(P, eps):
    e2 = eps * eps
    for i in range(P.shape[0]):
        s = oracle.normative_sqdist(P, P[i])
        if np.any(np.abs(s - e2) <= 1e-9 * e2):
            return False
    return True


@pytest.mark.parametrize(
    "seed,n,d,k,std,eps,min_samples",
    [
        (0, 400, 2, 5, 0.03, 0.03, 5),
        (1, 800, 2, 8, 0.02, 0.025, 4),
        (2, 600, 3, 6, 0.04, 0.06, 5),
        (3, 500, 3, 4, 0.05, 0.05, 10),
        (4, 300, 5, 3, 0.05, 0.12, 5),
        (5, 700, 2, 10, 0.01, 0.02, 1),
    ],
)
def test_matches_scikit_learn(seed, n, d, k, std, eps, min_samples):
    P = blobs(seed, n, d, k, std, 0.2)
    assert no_boundary_pairs(P, eps)
    got = dbscan(P, eps, min_samples)
    ref = sklearn_cluster.DBSCAN(eps=eps, min_samples=min_samples, algorithm="brute").fit(P)
    assert np.array_equal(got.labels, ref.labels_.astype(np.int32))
    core_ref = np.zeros(n, dtype=bool)
    core_ref[ref.core_sample_indices_] = True
    assert np.array_equal(got.core, core_ref)
    # the configurations exercise clusters, border points and noise
    assert got.labels.max() >= 1 and np.any(got.labels == -1) == (min_samples > 1)
    if min_samples > 1:
        assert np.any((got.labels >= 0) & ~got.core)


def test_isolated_points():
    P = np.arange(10, dtype=np.float64).reshape(-1, 1) * 10.0
    got = dbscan(P, 1.0, 2)
    assert np.all(got.labels == -1) and not got.core.any()
    got1 = dbscan(P, 1.0, 1)  # every point its own cluster, in index order
    assert np.array_equal(got1.labels, np.arange(10, dtype=np.int32))


def test_line_at_inclusive_boundary():
    P = np.arange(10, dtype=np.float64).reshape(-1, 1)
    got = dbscan(P, 1.0, 3)  # S = 1 = eps^2 counts: interior points have 3 neighbours
    assert np.array_equal(got.core, np.r_[False, [True] * 8, False])
    assert np.all(got.labels == 0)
    below = dbscan(P, np.nextafter(1.0, 0.0), 3)  # no neighbour but self
    assert np.all(below.labels == -1)


@pytest.mark.parametrize("flip", [False, True])
def test_shared_border_point(flip):
    # two clusters (cores at 1.0 and 3.0) both reach the border point 2.0
    xs = [0.0, 0.5, 1.0, 2.0, 3.0, 3.5, 4.0]
    if flip:
        xs = xs[::-1]
    P = np.array(xs).reshape(-1, 1)
    got = dbscan(P, 1.0, 4)
    pos = {x: i for i, x in enumerate(xs)}
    assert got.core[pos[1.0]] and got.core[pos[3.0]] and not got.core[pos[2.0]]
    a, b = got.labels[pos[1.0]], got.labels[pos[3.0]]
    assert a != b and {a, b} == {0, 1}
    # the cluster whose smallest core index comes first is numbered 0 and
    # keeps the shared border point
    assert got.labels[pos[2.0]] == 0
    assert got.labels[pos[2.0]] == (a if pos[1.0] < pos[3.0] else b)
    ref = sklearn_cluster.DBSCAN(eps=1.0, min_samples=4, algorithm="brute").fit(P)
    assert np.array_equal(got.labels, ref.labels_.astype(np.int32))


def test_min_samples_one_is_components():
    # components of the eps-graph: {0,1,2} chained, {3}, {4,5}
    P = np.array([[0.0], [0.9], [1.8], [5.0], [7.0], [7.5]])
    got = dbscan(P, 1.0, 1)
    assert np.array_equal(got.labels, np.array([0, 0, 0, 1, 2, 2], dtype=np.int32))


def test_from_neighbors_rejects_bad_min_samples():
    with pytest.raises(ValueError):
        dbscan_from_neighbors(np.array([0, 1]), np.array([0]), 0)


# ---- planted mistakes: each wrong variant must fail the pins above ----------
def _variant(kind):
    from collections import deque

    def run(row_ptr, col, min_samples):
        row_ptr = np.asarray(row_ptr, dtype=np.int64)
        col = np.asarray(col, dtype=np.int64)
        n = row_ptr.shape[0] - 1
        size = row_ptr[1:] - row_ptr[:-1]
        if kind == "strict":
            core = size > min_samples
        elif kind == "no_self":
            core = size - 1 >= min_samples
        else:
            core = size >= min_samples
        labels = np.full(n, -1, dtype=np.int32)
        nxt = 0
        for i in range(n):
            if labels[i] != -1 or not core[i]:
                continue
            labels[i] = nxt
            fr = deque([i])
            while fr:
                c = fr.popleft()
                for j in col[row_ptr[c]:row_ptr[c + 1]]:
                    if labels[j] == -1 or (kind == "last_wins" and not core[j]):
                        labels[j] = nxt
                        if core[j] or kind == "through_border":
                            fr.append(int(j))
            nxt += 1
        return labels

    return run


def _pins_hold(fn):
    for flip in (False, True):
        xs = [0.0, 0.5, 1.0, 2.0, 3.0, 3.5, 4.0]
        if flip:
            xs = xs[::-1]
        P = np.array(xs).reshape(-1, 1)
        nb = oracle.brute_radius(P, P, 1.0)
        ref = sklearn_cluster.DBSCAN(eps=1.0, min_samples=4, algorithm="brute").fit(P).labels_
        if not np.array_equal(fn(nb.row_ptr, nb.col, 4), ref):
            return False
    for args in [(0, 400, 2, 5, 0.03, 0.03, 5), (3, 500, 3, 4, 0.05, 0.05, 10)]:
        seed, n, d, k, std, eps, ms = args
        P = blobs(seed, n, d, k, std, 0.2)
        nb = oracle.brute_radius(P, P, eps)
        ref = sklearn_cluster.DBSCAN(eps=eps, min_samples=ms, algorithm="brute").fit(P).labels_
        if not np.array_equal(fn(nb.row_ptr, nb.col, ms), ref):
            return False
    return True


def test_pins_accept_the_oracle():
    assert _pins_hold(lambda rp, c, ms: dbscan_from_neighbors(rp, c, ms).labels)


@pytest.mark.parametrize("kind", ["strict", "no_self", "last_wins", "through_border"])
def test_pins_catch_planted_mistakes(kind):
    assert not _pins_hold(_variant(kind))
