"""Streaming inserts (snn_index_insert): after inserting batches into an
index, every query must return exactly the oracle's result over all points
inserted so far (ids in insertion order)."""

import sys

import numpy as np
import pytest

import oracle
from paper_2212_07679_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_07679_amd import binding

    return binding


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check_same(got, ref, what=""):
    row_ptr, col, dist = (t.cpu().numpy() for t in got[:3])
    assert np.array_equal(row_ptr, ref.row_ptr), what
    assert np.array_equal(col, ref.col), what
    rd = ref.dist.astype(np.float64)
    exact0 = rd == 0
    assert np.all(dist[exact0] == 0), what
    assert np.all(np.abs(dist.astype(np.float64) - rd)[~exact0] <= 1e-5 * rd[~exact0]), what


def check_view(idx, n):
    v = idx.view()
    key = v["key"].cpu().numpy()
    perm = v["perm"].cpu().numpy()
    assert v["n"] == n and np.all(np.diff(key) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(n))


@pytest.mark.parametrize("precision", ["auto", "mixed", "fp64"])
def test_inserts_match_oracle(B, precision):
    w = W.gmm16(n=36000, m=1500)
    parts = [w.P[:20000], w.P[20000:25000], w.P[25000:]]
    say(f"stream gmm16 small parts={[len(p) for p in parts]} precision={precision}")
    idx = B.Index(to_dev(parts[0]))
    for R in (1.5, 3.0):
        check_same(idx.query(to_dev(w.Q), R, precision=precision), oracle.brute_radius(parts[0], w.Q, R), "before")
    seen = parts[0]
    for p in parts[1:]:
        idx.insert(to_dev(p))
        seen = np.concatenate([seen, p])
        check_view(idx, seen.shape[0])
        for R in (1.5, 3.0):
            check_same(idx.query(to_dev(w.Q), R, precision=precision), oracle.brute_radius(seen, w.Q, R),
                       f"after {seen.shape[0]} R={R}")
    if precision == "auto":
        sub = seen[::3]  # every third row keeps the oracle's self-query short
        idx2 = B.Index(to_dev(sub[:5000]))
        idx2.insert(to_dev(sub[5000:]))
        check_same(idx2.query_self(3.0), oracle.brute_radius(sub, sub, 3.0), "self")


def test_inserts_beyond_the_original_extent(B):
    # new points far from the original data: the norm bound, the key error
    # bound and the screen constants must grow with them
    say("stream: far-away and duplicate inserts")
    g = np.random.default_rng([2212, 7679, 97])
    P0 = g.random((8000, 5)).astype(np.float32)
    far = (g.random((3000, 5)) * 40.0 + 25.0).astype(np.float32)
    dup = P0[g.choice(8000, 500, replace=False)]  # equal keys: existing rows stay first
    Q = np.concatenate([g.random((400, 5)), g.random((400, 5)) * 40.0 + 25.0]).astype(np.float32)
    idx = B.Index(to_dev(P0))
    idx.insert(to_dev(far))
    idx.insert(to_dev(dup))
    seen = np.concatenate([P0, far, dup])
    check_view(idx, seen.shape[0])
    for R, precision in ((0.2, "auto"), (0.2, "fp32"), (0.2, "mixed"), (3.0, "auto"), (3.0, "fp64")):
        check_same(idx.query(to_dev(Q), R, precision=precision), oracle.brute_radius(seen, Q, R),
                   f"R={R} {precision}")


def test_insert_float64_and_dbscan(B):
    say("stream: float64 rows, DBSCAN after inserts")
    w = W.blobs3d(n=9000, R=0.012, k=30)
    P = w.P.astype(np.float64)
    idx = B.Index(to_dev(P[:3000]))
    idx.insert(to_dev(P[3000:6000]))
    idx.insert(to_dev(P[6000:]))
    ref = oracle.dbscan(P, 0.012, 5)
    labels, core, k = idx.dbscan(0.012, 5)
    assert np.array_equal(labels.cpu().numpy(), ref.labels) and np.array_equal(core.cpu().numpy(), ref.core)
    assert k == int(ref.labels.max()) + 1


def test_insert_edge_cases(B):
    say("stream: empty insert, NaN insert leaves the index unchanged")
    g = np.random.default_rng([2212, 7679, 98])
    P0 = g.random((2000, 3))
    Q = g.random((100, 3))
    idx = B.Index(to_dev(P0))
    idx.insert(to_dev(np.zeros((0, 3))))
    bad = g.random((50, 3))
    bad[17, 1] = np.nan
    with pytest.raises(B.SnnError) as e:
        idx.insert(to_dev(bad))
    assert e.value.status == B.SNN_EINVAL
    assert idx.n == 2000  # the binding only counts successful inserts
    check_view(idx, 2000)
    check_same(idx.query(to_dev(Q), 0.1), oracle.brute_radius(P0, Q, 0.1), "unchanged")
    with pytest.raises(B.SnnError):
        idx.insert(to_dev(np.zeros((5, 4))))  # wrong d
    one = g.random((1, 3))
    idx.insert(to_dev(one))
    check_same(idx.query(to_dev(Q), 0.1), oracle.brute_radius(np.concatenate([P0, one]), Q, 0.1), "one more")
