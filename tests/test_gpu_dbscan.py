"""GPU DBSCAN (snn_dbscan on self-query lists) against the DBSCAN oracle.

Labels, core flags and the cluster count must equal the oracle's exactly
(the oracle runs its own brute-force neighbour lists).  At the full size of
the particle workload the labels are checked against the definition applied
to the GPU's own lists, whose rows are sampled against the oracle: core
flags from the row lengths, clusters against scipy's connected components
of the core graph, numbering by smallest core id, border points by the
smallest adjacent cluster.
"""

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


def check_against_oracle(B, P, eps, min_samples, precision="auto"):
    """Both GPU routes against the oracle: the fused one (self-query pairs
    clustered directly, symmetric and full scan) and snn_dbscan on the
    self-query's neighbour lists."""
    ref = oracle.dbscan(P, eps, min_samples)
    idx = B.Index(to_dev(P))
    row_ptr, col, _ = idx.query_self(eps, precision=precision)
    routes = {
        "fused": idx.dbscan(eps, min_samples, precision=precision),
        "fused, full scan": idx.dbscan(eps, min_samples, precision=precision, full_self_scan=True),
        "lists": B.dbscan_csr(row_ptr, col, min_samples, stream=idx.stream),
    }
    for name, (labels, core, k) in routes.items():
        labels, core = labels.cpu().numpy(), core.cpu().numpy()
        assert np.array_equal(core, ref.core), name
        assert np.array_equal(labels, ref.labels), name
        assert k == int(ref.labels.max()) + 1, name
    idx.close()
    return ref


@pytest.mark.parametrize(
    "n,k,eps,min_samples,dtype",
    [
        (6000, 30, 0.01, 5, np.float32),
        (8000, 40, 0.008, 5, np.float32),
        (6000, 20, 0.015, 10, np.float64),
        (6000, 30, 0.01, 1, np.float32),
        (6000, 30, 0.01, 60, np.float32),
    ],
)
def test_blobs_match_oracle(B, n, k, eps, min_samples, dtype):
    say(f"dbscan blobs3d n={n} k={k} eps={eps} min_samples={min_samples} {np.dtype(dtype).name}")
    w = W.blobs3d(n=n, R=eps, k=k)
    ref = check_against_oracle(B, w.P.astype(dtype), eps, min_samples)
    if 1 < min_samples < 60:
        # the case holds clusters, border points and noise
        assert ref.labels.max() >= 1 and np.any(ref.labels == -1) and np.any((ref.labels >= 0) & ~ref.core)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_every_screen_gives_the_same_clustering(B, precision):
    say(f"dbscan blobs3d small, precision={precision}")
    w = W.blobs3d(n=5000, R=0.012, k=25)
    check_against_oracle(B, w.P, 0.012, 5, precision=precision)


def test_lattice_ties_and_shared_border(B):
    say("dbscan lattice + shared border point")
    # unit lattice: distance 1 pairs sit exactly on the inclusive boundary
    P = W.lattice(0, 6, 2)
    check_against_oracle(B, P, 1.0, 5)
    check_against_oracle(B, P, float(np.nextafter(1.0, 0.0)), 2)
    for xs in ([0.0, 0.5, 1.0, 2.0, 3.0, 3.5, 4.0], [4.0, 3.5, 3.0, 2.0, 1.0, 0.5, 0.0]):
        check_against_oracle(B, np.array(xs).reshape(-1, 1), 1.0, 4)


def test_tiny_inputs(B):
    say("dbscan n=1, n=2")
    one = np.array([[0.5, 0.5]])
    check_against_oracle(B, one, 0.1, 1)
    check_against_oracle(B, one, 0.1, 2)
    two = np.array([[0.0, 0.0], [0.05, 0.0]])
    check_against_oracle(B, two, 0.1, 2)
    check_against_oracle(B, two, 0.01, 2)


def test_empty_lists(B):
    say("dbscan n=0 and rows with no entries")
    labels, core, k = B.dbscan_csr(torch.zeros(1, dtype=torch.int64, device="cuda:0"),
                                   torch.zeros(0, dtype=torch.int32, device="cuda:0"), 5)
    assert labels.numel() == 0 and core.numel() == 0 and k == 0
    # generic lists: an empty row is noise; with min_samples 1 a point with an
    # empty row is not core either
    rp = torch.tensor([0, 0, 2, 4, 4], dtype=torch.int64, device="cuda:0")
    col = torch.tensor([1, 2, 1, 2], dtype=torch.int32, device="cuda:0")
    labels, core, k = B.dbscan_csr(rp, col, 1)
    assert labels.cpu().tolist() == [-1, 0, 0, -1] and core.cpu().tolist() == [False, True, True, False] and k == 1


def test_rejects_malformed_lists(B):
    say("dbscan malformed lists")
    rp = torch.tensor([0, 2, 3], dtype=torch.int64, device="cuda:0")
    bad_col = torch.tensor([0, 5, 1], dtype=torch.int32, device="cuda:0")  # id 5 >= n = 2
    with pytest.raises(B.SnnError) as e:
        B.dbscan_csr(rp, bad_col, 2)
    assert e.value.status == B.SNN_EINVAL
    neg_col = torch.tensor([0, -1, 1], dtype=torch.int32, device="cuda:0")
    with pytest.raises(B.SnnError) as e:
        B.dbscan_csr(rp, neg_col, 2)
    assert e.value.status == B.SNN_EINVAL
    dec = torch.tensor([0, 3, 2, 3], dtype=torch.int64, device="cuda:0")  # row 1 ends before it starts
    col = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda:0")
    with pytest.raises(B.SnnError) as e:
        B.dbscan_csr(dec, col, 2)
    assert e.value.status == B.SNN_EINVAL


def test_deterministic(B):
    say("dbscan determinism")
    w = W.blobs3d(n=20000, R=0.006, k=60)
    X = to_dev(w.P)
    first = B.dbscan(X, 0.006, 5)
    for _ in range(3):
        again = B.dbscan(X, 0.006, 5)
        assert torch.equal(first[0], again[0]) and first[2] == again[2]
    idx = B.Index(X)
    labels, core, k, st = idx.dbscan(0.006, 5, stats=True)
    rp, col, _ = idx.query_self(0.006)
    assert st["nnz"] == int(rp[-1]) and torch.equal(labels, first[0])
    idx.close()


def test_fullsize_particles(B):
    """The particle workload at full size (n = 5e6, eps = R = 0.005,
    min_samples = 5, the setting of Section 6.4)."""
    sp = pytest.importorskip("scipy.sparse")
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    w = W.blobs3d()
    say(f"dbscan full-size blobs3d n={w.n} eps={w.R} min_samples=5")
    idx = B.Index(to_dev(w.P))
    row_ptr_d, col_d, _ = idx.query_self(w.R)
    labels_d, core_d, k = B.dbscan_csr(row_ptr_d, col_d, 5, stream=idx.stream)
    fused = idx.dbscan(w.R, 5)
    torch.cuda.synchronize()
    assert torch.equal(fused[0], labels_d) and torch.equal(fused[1], core_d) and fused[2] == k
    row_ptr, col = row_ptr_d.cpu().numpy(), col_d.cpu().numpy()
    labels, core = labels_d.cpu().numpy(), core_d.cpu().numpy()
    n = w.n
    # the lists themselves: sampled rows against the oracle
    g = np.random.default_rng(11)
    for i in g.choice(n, 20, replace=False):
        ref = oracle.brute_radius(w.P, w.P[i:i + 1], w.R)
        assert np.array_equal(col[row_ptr[i]:row_ptr[i + 1]], ref.col)
    lens = np.diff(row_ptr)
    assert np.array_equal(core, lens >= 5)
    # clusters = components of the core graph, numbered by smallest core id
    src = np.repeat(np.arange(n, dtype=np.int32), lens)
    keep = core[src] & core[col]
    A = sp.csr_matrix((np.ones(int(keep.sum()), dtype=np.int8), (src[keep], col[keep])), shape=(n, n))
    _, comp = csgraph.connected_components(A, directed=False)
    cidx = np.flatnonzero(core)
    ccomp = comp[cidx]
    first = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(first, ccomp, cidx)
    roots = np.sort(first[first < n])
    assert k == roots.size
    rank = np.full(n, -1, dtype=np.int64)
    rank[roots] = np.arange(roots.size)
    assert np.array_equal(labels[cidx], rank[first[ccomp]])
    # border points: smallest adjacent cluster; noise otherwise
    nc = ~core[src] & core[col]
    want = np.full(n, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(want, src[nc], labels[col[nc]].astype(np.int64))
    want[want == np.iinfo(np.int64).max] = -1
    assert np.array_equal(labels[~core], want[~core])
    say(f"  clusters={k} core={int(core.sum())} noise={int((labels == -1).sum())}")
    idx.close()
