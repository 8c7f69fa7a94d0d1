"""GPU parity for the Section 2 distances: row normalisation (bit-exact),
angular and cosine searches on normalised rows, and Manhattan searches
(every screen precision, out-of-sample and self-queries, lattice ties),
against the oracle."""

import math
import sys

import numpy as np
import pytest

import oracle
from oracle.metrics import brute_angular, brute_cosine, brute_l1, normalize_rows
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
    exact0 = ref.dist == 0
    assert np.all(dist[exact0] == 0), what
    rd = ref.dist.astype(np.float64)
    rel = np.abs(dist.astype(np.float64) - rd) / np.maximum(rd, 1e-300)
    assert np.all(rel[~exact0] <= 1e-5), what


@pytest.mark.parametrize("d", [1, 3, 100, 300])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_normalize_bit_exact(B, d, dtype):
    say(f"normalize d={d} {np.dtype(dtype).name}")
    g = np.random.default_rng([2212, 7679, 95, d])
    X = (g.standard_normal((3001, d)) * 10.0 ** g.integers(-20, 20, size=(3001, 1))).astype(dtype)
    Y = B.normalize_rows(to_dev(X)).cpu().numpy()
    assert np.array_equal(Y, normalize_rows(X))
    Xd = to_dev(X)
    B.normalize_rows(Xd, out=Xd)  # in place
    assert np.array_equal(Xd.cpu().numpy(), Y)


def test_normalize_rejects_zero_and_nan_rows(B):
    say("normalize rejects zero / NaN rows")
    for bad in (np.array([[1.0, 2.0], [0.0, 0.0]]), np.array([[1.0, np.nan]]), np.array([[np.inf, 1.0]])):
        with pytest.raises(B.SnnError) as e:
            B.normalize_rows(to_dev(bad))
        assert e.value.status == B.SNN_EINVAL


@pytest.mark.parametrize("precision", ["auto", "mixed", "fp64"])
def test_angular_and_cosine_search(B, precision):
    """The library takes the angle (or cosine distance) itself; the oracle
    decides by its own squared chord 2 - 2 cos(alpha) (or 2c)."""
    w = W.angular100(n=30000, m=700, k=3)
    say(f"angular100 small n={w.n} m={w.m} alpha={w.alpha} precision={precision}")
    Yp, Yq = normalize_rows(w.P), normalize_rows(w.Q)
    Xd = B.normalize_rows(to_dev(w.P))
    Qd = B.normalize_rows(to_dev(w.Q))
    idx = B.Index(Xd)
    ref = brute_angular(Yp, Yq, w.alpha)
    assert ref.row_ptr[-1] > w.m  # neighbours beyond a handful
    check_same(idx.query(Qd, w.alpha, precision=precision, metric="angular"), ref, "angular")
    c = 1.0 - math.cos(w.alpha) * 1.01
    check_same(idx.query(Qd, c, precision=precision, metric="cosine"), brute_cosine(Yp, Yq, c), "cosine")
    # self-queries (symmetric and full scans) and clustering with the angular neighbourhood
    Ys = Yp[:6000]
    idx2 = B.Index(to_dev(Ys))
    refs = brute_angular(Ys, Ys, w.alpha)
    check_same(idx2.query_self(w.alpha, precision=precision, metric="angular"), refs, "angular self")
    check_same(idx2.query_self(w.alpha, precision=precision, metric="angular", full_self_scan=True), refs,
               "angular self full")
    refd = oracle.dbscan_from_neighbors(refs.row_ptr, refs.col, 5)
    labels, core, k = idx2.dbscan(w.alpha, 5, precision=precision, metric="angular")
    assert np.array_equal(labels.cpu().numpy(), refd.labels) and np.array_equal(core.cpu().numpy(), refd.core)


def test_angular_boundary_and_errors(B):
    """Unit vectors 7 degrees apart on a circle: an angle of exactly 14
    degrees between the radii of two points decides by the squared chord."""
    say("angular on a circle, errors")
    ang = np.arange(60) * math.radians(7.0)
    Y = normalize_rows(np.stack([np.cos(ang), np.sin(ang)], axis=1))
    idx = B.Index(to_dev(Y))
    for a_deg in (0.0, 6.9, 14.0, 20.0, 180.0):
        a = math.radians(a_deg)
        for precision in ("auto", "mixed", "fp64", "fp32"):
            check_same(idx.query(to_dev(Y), a, precision=precision, metric="angular"), brute_angular(Y, Y, a),
                       f"angle {a_deg} {precision}")
    with pytest.raises(B.SnnError) as e:
        idx.query(to_dev(Y), math.pi * 1.01, metric="angular")
    assert e.value.status == B.SNN_EINVAL
    with pytest.raises(B.SnnError) as e:
        idx.query(to_dev(Y), -0.1, metric="cosine")
    assert e.value.status == B.SNN_EINVAL


@pytest.mark.parametrize("precision", ["auto", "mixed", "fp32", "fp64"])
@pytest.mark.parametrize("d", [1, 3, 8, 16])
def test_manhattan_low_d(B, precision, d):
    g = np.random.default_rng([2212, 7679, 96, d])
    P = g.random((20000, d)).astype(np.float32)
    Q = g.random((1500, d)).astype(np.float32)
    # about 8 expected neighbours: the 1-ball of radius R has volume (2R)^d / d!
    R = 0.5 * (8.0 * math.factorial(d) / P.shape[0]) ** (1.0 / d) * (1.2 if d > 3 else 1.0)
    say(f"manhattan d={d} R={R:.3f} precision={precision}")
    idx = B.Index(to_dev(P))
    ref = brute_l1(P, Q, R)
    assert ref.row_ptr[-1] > 0
    check_same(idx.query(to_dev(Q), R, precision=precision, metric="l1"), ref, "l1")


@pytest.mark.parametrize("precision", ["auto", "fp64"])
def test_manhattan_high_d_and_self(B, precision):
    w = W.gmm16(n=40000, m=2000)
    R = 4.5
    say(f"manhattan gmm16 small R={R} precision={precision}")
    idx = B.Index(to_dev(w.P))
    check_same(idx.query(to_dev(w.Q), R, precision=precision, metric="l1"), brute_l1(w.P, w.Q, R), "l1 gmm16")
    Ps = w.P[:12000]
    idx2 = B.Index(to_dev(Ps))
    ref = brute_l1(Ps, Ps, R)
    check_same(idx2.query_self(R, precision=precision, metric="l1"), ref, "l1 self")
    check_same(idx2.query_self(R, precision=precision, metric="l1", full_self_scan=True), ref, "l1 self full")


def test_manhattan_lattice_ties(B):
    say("manhattan lattice ties")
    P = W.lattice(-6, 6, 3)
    Q = W.lattice(-2, 2, 3)
    for R in (1.0, 3.0, 5.0):
        for precision in ("auto", "mixed", "fp64"):
            check_same(B.Index(to_dev(P)).query(to_dev(Q), R, precision=precision, metric="l1"), brute_l1(P, Q, R),
                       f"lattice R={R} {precision}")


def test_manhattan_dbscan(B):
    say("dbscan with the Manhattan neighbourhood")
    w = W.blobs3d(n=6000, R=0.012, k=30)
    ref_nb = brute_l1(w.P, w.P, 0.012)
    ref = oracle.dbscan_from_neighbors(ref_nb.row_ptr, ref_nb.col, 5)
    labels, core, k = B.Index(to_dev(w.P)).dbscan(0.012, 5, metric="l1")
    assert np.array_equal(labels.cpu().numpy(), ref.labels) and np.array_equal(core.cpu().numpy(), ref.core)
    assert k == int(ref.labels.max()) + 1


def test_metric_argument_errors(B):
    idx = B.Index(to_dev(np.zeros((4, 2))))
    with pytest.raises(B.SnnError):
        idx.query(to_dev(np.zeros((1, 2))), 1.0, metric="linf")
    opts = B.snn_options(2, 0, 0, 0, 0, 7)
    csr = B.snn_csr(0, 0, 0, 0, 0)
    rp = torch.empty(2, dtype=torch.int64, device="cuda:0")
    csr.row_ptr = rp.data_ptr()
    import ctypes

    st = B.lib().snn_query(idx._h, ctypes.c_void_p(to_dev(np.zeros((1, 2))).data_ptr()), 1, 1.0, ctypes.byref(opts),
                           ctypes.byref(csr), None)
    assert st == B.SNN_EINVAL
