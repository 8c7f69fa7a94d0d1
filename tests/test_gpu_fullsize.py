"""GPU parity at the full workload sizes, in the configuration bench.py times.

The oracle cannot finish a full run in seconds, so each test checks seeded
sampled rows one by one against the brute-force oracle (bit-exact ids and
row lengths, distances within 1e-5 relative) and checks properties that hold
at any size on the whole output: row pointers monotone and consistent with
nnz, ids in range and strictly ascending within every row, every distance
within R, and the self match present in every self-query row.
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


def check_whole(row_ptr, col, dist, n, R, self_query):
    m = row_ptr.shape[0] - 1
    assert row_ptr[0] == 0 and np.all(np.diff(row_ptr) >= 0)
    assert row_ptr[-1] == col.shape[0] == dist.shape[0]
    if col.size:
        assert col.min() >= 0 and col.max() < n
        # strictly ascending inside each row: a drop is allowed only at row starts
        drops = np.flatnonzero(np.diff(col.astype(np.int64)) <= 0) + 1
        starts = np.zeros(col.shape[0], dtype=bool)
        starts[row_ptr[1:-1][row_ptr[1:-1] < col.shape[0]]] = True
        assert np.all(starts[drops]), "ids not strictly ascending within a row"
        assert np.all(dist >= 0) and np.all(dist <= np.float32(R) * (1 + 1e-6))
    if self_query:
        lens = np.diff(row_ptr)
        assert np.all(lens >= 1), "a self-query row lacks its own point"
        rows = np.repeat(np.arange(m), lens)
        hit = np.zeros(m, dtype=bool)
        hit[rows[col == rows]] = True
        assert np.all(hit), "self match missing"


_ORACLE_INDEX = {}


def oracle_rows(P, Q, R, rows, key):
    """The oracle's rows for the given queries: the CPU SNN (Algorithms 1-2,
    pinned equal to brute force by eq. (lower)) on a cached oracle index."""
    if key not in _ORACLE_INDEX:
        _ORACLE_INDEX.clear()
        _ORACLE_INDEX[key] = oracle.build_index(P)
    nb, _ = oracle.snn_query(_ORACLE_INDEX[key], Q[rows], R)
    return nb


def check_rows(row_ptr, col, dist, P, Q, R, rows, key=None):
    if key is None:
        ref = oracle.brute_radius(P, Q[rows], R, max_block_elems=1 << 25)
    else:
        ref = oracle_rows(P, Q, R, rows, key)
    for k, r in enumerate(rows):
        a, b = row_ptr[r], row_ptr[r + 1]
        ra, rb = ref.row_ptr[k], ref.row_ptr[k + 1]
        assert b - a == rb - ra, f"row {r}: {b - a} neighbours, oracle {rb - ra}"
        assert np.array_equal(col[a:b], ref.col[ra:rb]), f"row {r}: ids differ"
        rd, gd = ref.dist[ra:rb], dist[a:b]
        z = rd == 0
        assert np.all(gd[z] == 0)
        assert np.all(np.abs(gd[~z] - rd[~z]) <= 1e-5 * rd[~z]), f"row {r}: distance"


def sample_rows(m, count, seed, extra=()):
    g = np.random.default_rng([2212, 7679, 99, seed])
    rows = set(g.choice(m, size=min(count, m), replace=False).tolist())
    rows.update(int(r) for r in extra if 0 <= r < m)
    return np.array(sorted(rows), dtype=np.int64)


def run(B, w, prec, rows_count, seed, dense_rows=0, nonempty=False, key=None):
    say(f"full-size {w.name}: n={w.n} d={w.d} m={w.m} R={w.R} precision={prec}")
    idx = B.Index(to_dev(w.P))
    Qd = None if w.Q is None else to_dev(w.Q)
    out = idx.query_self(w.R, precision=prec, stats=True) if Qd is None else idx.query(Qd, w.R, precision=prec, stats=True)
    torch.cuda.synchronize()
    row_ptr, col, dist = (t.cpu().numpy() for t in out[:3])
    st = out[3]
    say(f"  nnz={row_ptr[-1]} precision_used={B.PRECISION_NAMES[st['precision_used']]} terms={st['terms_used']} "
        f"window pairs={st['pairs_window']} rechecked={st['pairs_recheck']}")
    assert st["nnz"] == row_ptr[-1]
    assert st["pairs_executed"] >= st["pairs_window"]
    check_whole(row_ptr, col, dist, w.n, w.R, w.Q is None)
    extra = ()
    if dense_rows:
        lens = np.diff(row_ptr)
        extra = np.argsort(lens)[-dense_rows:]  # the longest rows
    if nonempty:  # every row with a neighbour, beside the sample
        extra = np.concatenate([np.asarray(extra, dtype=np.int64), np.flatnonzero(np.diff(row_ptr) > 0)])
    rows = sample_rows(w.m, rows_count, seed, extra)
    check_rows(row_ptr, col, dist, w.P, w.queries, w.R, rows, key)
    say(f"  {rows.size} rows ({'all non-empty rows and ' if nonempty else ''}a seeded sample) match the oracle")
    return st, out


def test_gmm16_full(B):
    """The headline workload in the bench's configuration: the mixed and the
    plain float64 screens give byte-identical CSR arrays over all 1e5 rows,
    and every non-empty row plus 5000 sampled rows equal the oracle's."""
    w = W.gmm16()
    outs = {}
    for prec in ("mixed", "fp64"):
        st, out = run(B, w, prec, 5000, 1, nonempty=True, key="gmm16")
        assert B.PRECISION_NAMES[st["precision_used"]] == prec
        outs[prec] = out
    for a, b in zip(outs["mixed"][:3], outs["fp64"][:3]):
        assert torch.equal(a, b), "mixed and float64 screens differ"


def test_gmm16_full_wide_radius(B):
    # the headline data with a radius that yields many neighbours per query
    w = W.gmm16(R=4.0)
    run(B, w, "mixed", 1000, 2, dense_rows=5, key="gmm16")


def test_uniform2d_full_auto(B):
    w = W.uniform2d()
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    idx = B.Index(to_dev(w.P))
    for prec in ("auto", "fp64"):
        row_ptr, col, dist = (t.cpu().numpy() for t in idx.query(to_dev(w.Q), w.R, precision=prec)[:3])
        assert np.array_equal(row_ptr, ref.row_ptr) and np.array_equal(col, ref.col)
        assert np.all(np.abs(dist - ref.dist) <= 1e-5 * ref.dist)


def test_blobs3d_full(B):
    w = W.blobs3d()
    run(B, w, "auto", 200, 3, dense_rows=5)


def test_gmm128z_full(B):
    w = W.gmm128z()
    run(B, w, "auto", 200, 4, key="gmm128z")
