"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Index sets and row pointers must be bit-identical to the oracle; distances
within 1e-5 relative (exactly 0 for S = 0).  Sizes span several tiles and
work units with ragged tails.
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


def check_same(got, ref, what=""):
    row_ptr, col, dist = (t.cpu().numpy() for t in got[:3])
    assert row_ptr.shape == ref.row_ptr.shape, what
    bad = np.flatnonzero(row_ptr != ref.row_ptr)
    assert bad.size == 0, f"{what}: row_ptr differs first at {bad[:5]}"
    assert np.array_equal(col, ref.col), f"{what}: col differs"
    zero = ref.dist == 0
    assert np.all(dist[zero] == 0), what
    nz = ~zero
    rel = np.abs(dist[nz] - ref.dist[nz]) / ref.dist[nz]
    assert np.all(rel <= 1e-5), f"{what}: max rel dist err {rel.max()}"


PRECS = ["fp64", "mixed", "fp16", "fp32", "auto"]


@pytest.mark.parametrize("terms", [1, 3])
@pytest.mark.parametrize("R", [1.5, 4.0])
def test_mixed_terms_gmm16(B, terms, R):
    w = W.gmm16(n=40_000, m=2_000, R=R)
    say(f"mixed terms={terms} gmm16 n={w.n} m={w.m} R={R}")
    ref, _ = oracle.snn_query(oracle.build_index(w.P), w.Q, w.R)
    idx = B.Index(to_dev(w.P))
    got = idx.query(to_dev(w.Q), w.R, precision="mixed", terms=terms, stats=True)
    check_same(got, ref, f"mixed terms={terms} R={R}")
    st = got[3]
    assert st["terms_used"] == terms and st["precision_used"] == 1
    assert st["pairs_recheck"] >= st["nnz"]


@pytest.mark.parametrize("terms", [1, 3])
def test_mixed_self_gmm128(B, terms):
    w = W.gmm128z(n=12_000, R=4.0)
    say(f"mixed self terms={terms} gmm128z n={w.n}")
    ref, _ = oracle.snn_query(oracle.build_index(w.P), w.P, w.R)
    idx = B.Index(to_dev(w.P))
    # d = 128: three bf16 terms need 384-wide rows, beyond the packed limit
    if terms == 3:
        with pytest.raises(B.SnnError) as e:
            idx.query_self(w.R, precision="mixed", terms=3)
        assert e.value.status == B.SNN_ENOTSUP
        return
    check_same(idx.query_self(w.R, precision="mixed", terms=1), ref, "gmm128z self")
    # a radius with many positives
    ref2, _ = oracle.snn_query(oracle.build_index(w.P), w.P[:3000], 9.0)
    check_same(idx.query(to_dev(w.P[:3000]), 9.0, precision="mixed", terms=1), ref2, "gmm128z R=9")


@pytest.mark.parametrize("prec", PRECS)
def test_uniform2d_full(B, prec):
    w = W.uniform2d()
    say(f"uniform2d n={w.n} m={w.m} R={w.R} prec={prec}")
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    idx = B.Index(to_dev(w.P))
    got = idx.query(to_dev(w.Q), w.R, precision=prec, stats=True)
    check_same(got, ref, "uniform2d")
    st = got[3]
    o2, ost = oracle.snn_query(oracle.build_index(w.P), w.Q, w.R)
    assert st["nnz"] == ref.row_ptr[-1]
    # the GPU window is at least the exact-arithmetic window and close to it
    assert st["pairs_window"] >= 0.99 * ost["pairs_window"]
    assert st["pairs_window"] <= 1.05 * ost["pairs_window"] + 1000
    # the screen scans tile windows (a superset of every query's window) for
    # whole query blocks
    assert st["pairs_executed"] >= st["pairs_window"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("R", [1.5, 3.0])
def test_gmm16_small(B, prec, R):
    w = W.gmm16(n=30_000, m=3_000, R=R)
    say(f"gmm16 n={w.n} m={w.m} R={R} prec={prec}")
    idx_o = oracle.build_index(w.P)
    ref, _ = oracle.snn_query(idx_o, w.Q, w.R)
    idx = B.Index(to_dev(w.P))
    got = idx.query(to_dev(w.Q), w.R, precision=prec)
    check_same(got, ref, f"gmm16 R={R}")


@pytest.mark.parametrize("prec", PRECS)
def test_self_query_blobs(B, prec):
    w = W.blobs3d(n=20_000, R=0.02)
    say(f"blobs3d self n={w.n} R={w.R} prec={prec}")
    ref, _ = oracle.snn_query(oracle.build_index(w.P), w.P, w.R)
    idx = B.Index(to_dev(w.P))
    got = idx.query_self(w.R, precision=prec)
    check_same(got, ref, "blobs3d self")


@pytest.mark.parametrize("d", [1, 3, 5, 8, 13, 32, 37, 70, 129, 300, 1024])
def test_dims(B, d):
    g = np.random.default_rng(100 + d)
    n, m = 3000, 257
    P = g.standard_normal((n, d)).astype(np.float32)
    Q = np.concatenate([P[:100], g.standard_normal((m - 100, d)).astype(np.float32)])
    R = float(np.sqrt(d) * 0.6)
    say(f"dims d={d} n={n} m={m} R={R}")
    ref = oracle.brute_radius(P, Q, R)
    idx = B.Index(to_dev(P))
    for prec in PRECS:
        if (prec == "fp32" and d > 16) or (prec in ("mixed", "fp16") and d > 128):
            with pytest.raises(B.SnnError) as e:
                idx.query(to_dev(Q), R, precision=prec)
            assert e.value.status == B.SNN_ENOTSUP
            continue
        check_same(idx.query(to_dev(Q), R, precision=prec), ref, f"d={d} {prec}")


def test_edge_cases(B):
    say("edge cases")
    g = np.random.default_rng(7)
    P = g.random((500, 3))
    idx = B.Index(to_dev(P))
    # m = 0
    rp, col, dist = idx.query(to_dev(np.zeros((0, 3))), 0.1)
    assert rp.cpu().tolist() == [0] and col.numel() == 0
    # R = 0 with exact duplicates
    P2 = np.concatenate([P, P[:50]])
    idx2 = B.Index(to_dev(P2))
    check_same(idx2.query_self(0.0), oracle.brute_radius(P2, P2, 0.0), "R=0 duplicates")
    # n = 1
    idx1 = B.Index(to_dev(P[:1]))
    check_same(idx1.query(to_dev(P[:5]), 0.3), oracle.brute_radius(P[:1], P[:5], 0.3), "n=1")
    # every point a neighbour of every query: long rows (> 4096 needs merges)
    P3 = g.random((6000, 2))
    idx3 = B.Index(to_dev(P3))
    Q3 = P3[:70]
    check_same(idx3.query(to_dev(Q3), 2.0), oracle.brute_radius(P3, Q3, 2.0), "all neighbours")
    # rows of 17..64 and 65..4096 entries
    check_same(idx3.query(to_dev(Q3), 0.06), oracle.brute_radius(P3, Q3, 0.06), "medium rows")
    check_same(idx3.query(to_dev(Q3), 0.4), oracle.brute_radius(P3, Q3, 0.4), "long rows")


@pytest.mark.parametrize("prec", PRECS)
def test_lattice_ties(B, prec):
    say(f"lattice ties {prec}")
    P = W.lattice(-12, 12, 2)
    Q = P[::13]
    idx = B.Index(to_dev(P))
    check_same(idx.query(to_dev(Q), 5.0, precision=prec), oracle.brute_radius(P, Q, 5.0), "lattice R=5")
    P3 = W.lattice(-5, 5, 3).astype(np.float32)
    idx3 = B.Index(to_dev(P3))
    check_same(idx3.query_self(3.0, precision=prec), oracle.brute_radius(P3, P3, 3.0), "3-D lattice self")


@pytest.mark.parametrize("prec", PRECS)
def test_far_from_origin(B, prec):
    # near-duplicates far from the mean: large ||x|| against a tiny radius
    say(f"far from origin {prec}")
    g = np.random.default_rng(8)
    P = np.concatenate([1e4 + g.standard_normal((2000, 4)) * 1e-3, -1e4 + g.standard_normal((2000, 4)) * 1e-3])
    Q = P[::9] + 1e-4 * g.standard_normal((P[::9].shape[0], 4))
    idx = B.Index(to_dev(P))
    check_same(idx.query(to_dev(Q), 2e-3, precision=prec), oracle.brute_radius(P, Q, 2e-3), "far")


def test_determinism(B):
    say("determinism")
    w = W.gmm16(n=20_000, m=1_000, R=3.0)
    idx = B.Index(to_dev(w.P))
    a = [t.cpu().numpy().tobytes() for t in idx.query(to_dev(w.Q), w.R)]
    b = [t.cpu().numpy().tobytes() for t in idx.query(to_dev(w.Q), w.R)]
    assert a == b


def test_overflow_and_retry(B):
    say("overflow")
    w = W.uniform2d(n=5000, m=500, R=0.05)
    idx = B.Index(to_dev(w.P))
    with pytest.raises(B.SnnError) as e:
        idx.query(to_dev(w.Q), w.R, nnz_cap=10)
    assert e.value.status == B.SNN_EOVERFLOW
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    check_same(idx.query(to_dev(w.Q), w.R), ref, "after retry")


def test_nan_rejected(B):
    say("nan")
    P = np.random.default_rng(1).random((100, 3)).astype(np.float32)
    Pn = P.copy()
    Pn[17, 1] = np.nan
    with pytest.raises(B.SnnError) as e:
        B.Index(to_dev(Pn))
    assert e.value.status == B.SNN_EINVAL
    idx = B.Index(to_dev(P))
    Q = P[:5].copy()
    Q[2, 0] = np.inf
    with pytest.raises(B.SnnError) as e:
        idx.query(to_dev(Q), 0.1)
    assert e.value.status == B.SNN_EINVAL
    with pytest.raises(B.SnnError):
        idx.query(to_dev(P[:5]), -1.0)


@pytest.mark.parametrize("d", [3, 16, 40, 129, 300, 1024])
def test_index_internals(B, d):
    # every shape of the row kernels: one to eight elements per lane and
    # pass, several passes per row (d > 128), the centre and direction held
    # in registers (d <= 128) or in LDS (up to the largest d, 1024)
    say(f"index internals d={d}")
    if d == 16:
        P = W.gmm16(n=50_000, m=10, R=1.5).P
    else:
        g = np.random.default_rng([2212, 7679, 101, d])
        scale = np.linspace(1.0, 2.0, d)
        scale[d // 3] = 3.0
        P = (g.standard_normal((20_000, d)) * scale + 5.0).astype(np.float32)
    idx = B.Index(to_dev(P))
    v = idx.view()
    P = P.astype(np.float64)
    mu = P.mean(0)
    assert np.allclose(v["mu"].cpu().numpy(), mu, rtol=1e-12, atol=1e-12)
    vv = v["v"].cpu().numpy()
    assert abs(np.linalg.norm(vv) - 1) < 1e-12
    X = P - mu
    C = X.T @ X
    lam = np.linalg.eigvalsh(C)
    assert vv @ C @ vv >= (1 - 1e-6) * lam[-1]  # Rayleigh quotient of the power iteration
    key = v["key"].cpu().numpy()
    perm = v["perm"].cpu().numpy()
    assert np.all(np.diff(key) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(P.shape[0]))
    alpha = X[perm] @ vv
    assert np.all(np.abs(key - alpha) <= v["key_eps"])


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 16, 64, 65, 100, 128, 129, 200])
def test_power_iteration_widths(B, d):
    # every form of the direction solve (Jacobi rotations for d <= 4; the
    # power iteration in one wavefront, with C in LDS for 64 < d <= 128, or
    # C through the caches above): unit v along the top eigenvector of a
    # spectrum with a clear gap, Rayleigh quotient at the top
    say(f"power iteration d={d}")
    g = np.random.default_rng([2212, 7679, 99, d])
    scale = np.linspace(1.0, 2.0, d)
    scale[d // 3] = 3.0
    P = (g.standard_normal((20_000, d)) * scale).astype(np.float32)
    v = B.Index(to_dev(P)).view()
    X = P.astype(np.float64) - P.astype(np.float64).mean(0)
    C = X.T @ X
    lam, vec = np.linalg.eigh(C)
    vv = v["v"].cpu().numpy()
    assert abs(np.linalg.norm(vv) - 1) < 1e-12
    assert vv @ C @ vv >= (1 - 1e-9) * lam[-1]
    assert abs(vv @ vec[:, -1]) >= 1 - 1e-6
    assert 1 <= v["power_iters"] <= 500


@pytest.mark.parametrize("d", [2, 3])
def test_direction_near_degenerate(B, d):
    # two nearly equal top eigenvalues (the uniform square and cube): the
    # Jacobi solve still returns a top eigenvector, in a few sweeps
    say(f"direction near-degenerate d={d}")
    g = np.random.default_rng([2212, 7679, 102, d])
    P = g.random((50_000, d)).astype(np.float32)
    v = B.Index(to_dev(P)).view()
    X = P.astype(np.float64) - P.astype(np.float64).mean(0)
    C = X.T @ X
    lam = np.linalg.eigvalsh(C)
    vv = v["v"].cpu().numpy()
    assert vv @ C @ vv >= (1 - 1e-12) * lam[-1]
    assert v["power_iters"] <= 10


@pytest.mark.parametrize("n,bits", [(1, (0, 32)), (1000, (0, 32)), (100_003, (0, 32)), (70_000, (8, 32)),
                                    (5000, (0, 3)), (30_001, (0, 9)), (30_001, (4, 24)), (4097, (5, 16)),
                                    (2_500_003, (0, 32))])
def test_radix_sort(B, n, bits):
    say(f"radix sort n={n} bits={bits}")
    g = np.random.default_rng(n)
    k = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    k[: n // 3] = k[n // 3 : 2 * (n // 3)]  # many equal keys: stability matters
    vals = np.arange(n, dtype=np.uint32)
    kt = to_dev(k.view(np.int32))
    vt = to_dev(vals.view(np.int32))
    B.sort_pairs_u32(kt, vt, *bits)
    torch.cuda.synchronize()
    mask = np.uint32(((1 << (bits[1] - bits[0])) - 1) << bits[0]) if bits[1] - bits[0] < 32 else np.uint32(0xFFFFFFFF)
    order = np.argsort(k & mask, kind="stable")
    assert np.array_equal(vt.cpu().numpy().view(np.uint32), vals[order])
    assert np.array_equal(kt.cpu().numpy().view(np.uint32), k[order])


def test_auto_policy(B):
    # the plan follows the width of each screen's rounding band against R^2
    say("auto policy")
    w = W.blobs3d(n=30_000, R=0.005)
    idx = B.Index(to_dev(w.P))
    st = idx.query_self(w.R, stats=True)[3]
    assert B.PRECISION_NAMES[st["precision_used"]] == "fp32"  # bf16 band ~ R^2 for d = 3, tiny R
    w2 = W.gmm16(n=30_000, m=500, R=1.5)
    idx2 = B.Index(to_dev(w2.P))
    st2 = idx2.query(to_dev(w2.Q), w2.R, stats=True)[3]
    assert B.PRECISION_NAMES[st2["precision_used"]] == "fp16" and st2["terms_used"] == 1  # fp16 band < R^2
    st2b = idx2.query(to_dev(w2.Q), 0.9, stats=True)[3]
    assert B.PRECISION_NAMES[st2b["precision_used"]] == "mixed" and st2b["terms_used"] == 3  # fp16 band > R^2
    w3 = W.gmm128z(n=5_000, R=4.0)
    idx3 = B.Index(to_dev(w3.P))
    st3 = idx3.query_self(w3.R, stats=True)[3]
    assert B.PRECISION_NAMES[st3["precision_used"]] == "fp16" and st3["terms_used"] == 1


@pytest.mark.parametrize("prec", ["fp32", "mixed", "fp16", "fp64"])
def test_symmetric_self_scan(B, prec):
    # each unordered pair scanned once and reported in both rows: identical
    # output to the full scan, with about half the window pairs
    say(f"symmetric self scan {prec}")
    w = W.blobs3d(n=30_000, R=0.03, seed=11)
    ref, _ = oracle.snn_query(oracle.build_index(w.P), w.P, w.R)
    idx = B.Index(to_dev(w.P))
    half = idx.query_self(w.R, precision=prec, stats=True)
    full = idx.query_self(w.R, precision=prec, stats=True, full_self_scan=True)
    check_same(half, ref, f"symmetric {prec}")
    check_same(full, ref, f"full {prec}")
    hw, fw = half[3]["pairs_window"], full[3]["pairs_window"]
    assert 0.45 * fw < hw < 0.6 * fw, (hw, fw)


@pytest.mark.parametrize("prec", ["fp32", "mixed", "fp16", "fp64"])
def test_dense_self_output(B, prec):
    # many neighbours per row: survivor staging drains, wave/block row sorts
    say(f"dense self {prec}")
    w = W.blobs3d(n=40_000, R=0.03, seed=9)
    ref, _ = oracle.snn_query(oracle.build_index(w.P), w.P, w.R)
    assert ref.row_ptr[-1] > 20 * w.n
    idx = B.Index(to_dev(w.P))
    check_same(idx.query_self(w.R, precision=prec), ref, f"dense self {prec}")


@pytest.mark.parametrize("precision", ["mixed", "fp16", "fp32", "fp64"])
@pytest.mark.parametrize("tile_c", [32, 96, 1024])
def test_small_work_units(B, precision, tile_c):
    """Many work units per tile (and chunk ends inside windows) for every screen."""
    w = W.gmm16(n=30_000, m=900, R=3.0)
    say(f"small work units: tile_c={tile_c} precision={precision}")
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    idx = B.Index(to_dev(w.P))
    check_same(idx.query(to_dev(w.Q), w.R, precision=precision, tile_c=tile_c), ref, f"tile_c={tile_c}")
    selfw = w.P[:6000]
    ref_s = oracle.brute_radius(selfw, selfw, w.R)
    idx_s = B.Index(to_dev(selfw))
    check_same(idx_s.query_self(w.R, precision=precision, tile_c=tile_c), ref_s, f"self tile_c={tile_c}")
