"""Repeated query calls replayed from captured graphs.

A call repeated with the same inputs, outputs and workspace is captured on
its second occurrence and replayed afterwards.  Each test calls the C ABI
with fixed output buffers several times in a row, with other calls on the
same index and plain device work in between, and checks every call against
the oracle (Algorithm 2 pinned equal to brute force): the replays must see
the current contents of the query buffer, and the calls in between must not
disturb them.
"""

import ctypes
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


class FixedOut:
    """CSR output buffers that stay at one address across calls."""

    def __init__(self, m, cap):
        self.row_ptr = torch.empty(m + 1, dtype=torch.int64, device="cuda:0")
        self.col = torch.empty(cap, dtype=torch.int32, device="cuda:0")
        self.dist = torch.empty(cap, dtype=torch.float32, device="cuda:0")
        self.cap = cap

    def call(self, B, idx, Q, m, R, precision, self_query=False, stats=True):
        opts = idx._opts(precision, 0, 0, 0)
        csr = B.snn_csr(self.row_ptr.data_ptr(), self.col.data_ptr(), self.dist.data_ptr(), self.cap, 0)
        st = B.snn_stats()
        # the library's stream is separate from torch's: order the buffer
        # writes made on torch's stream before the call
        torch.cuda.synchronize()
        if self_query:
            status = B.lib().snn_query_self(idx._h, float(R), ctypes.byref(opts), ctypes.byref(csr),
                                            ctypes.byref(st) if stats else None)
        else:
            status = B.lib().snn_query(idx._h, ctypes.c_void_p(Q.data_ptr()), m, float(R), ctypes.byref(opts),
                                       ctypes.byref(csr), ctypes.byref(st) if stats else None)
        assert status == 0, f"status {status}"
        nnz = int(csr.nnz)
        return (self.row_ptr.cpu().numpy().copy(), self.col[:nnz].cpu().numpy().copy(),
                self.dist[:nnz].cpu().numpy().copy())


def check(got, ref, what):
    row_ptr, col, dist = got
    assert np.array_equal(row_ptr, ref.row_ptr), f"{what}: row_ptr"
    assert np.array_equal(col, ref.col), f"{what}: col"
    z = ref.dist == 0
    assert np.all(dist[z] == 0), what
    assert np.all(np.abs(dist[~z] - ref.dist[~z]) <= 1e-5 * ref.dist[~z]), f"{what}: dist"


@pytest.fixture(scope="module")
def gmm():
    """gmm16-shaped set (rows of up to ~128 neighbours at R = 3.5), a second
    query set near the first, and the oracle's lists at R = 3.5 and 3.0."""
    w = W.gmm16(n=15_000, m=1_500, R=3.5)
    g = np.random.default_rng([2212, 7679, 31])
    Q2 = (w.Q + g.normal(0, 0.05, w.Q.shape)).astype(np.float32)
    refs = {(q, R): oracle.brute_radius(w.P, Q, R) for q, Q in ((1, w.Q), (2, Q2)) for R in (3.5, 3.0)}
    return w, Q2, refs


@pytest.mark.parametrize("precision", ["auto", "mixed", "fp64"])
def test_replays_out_of_sample(B, gmm, precision):
    w, Q2, refs = gmm
    say(f"graph replays: gmm16 n={w.n} m={w.m} R={w.R} precision={precision} nnz={refs[(1, 3.5)].col.size}")
    idx = B.Index(to_dev(w.P))
    Qd = to_dev(w.Q)
    out = FixedOut(w.m, max(r.col.size for r in refs.values()) + 1024)
    other = FixedOut(w.m, max(r.col.size for r in refs.values()) + 1024)
    for k in range(6):
        if k == 4:  # new contents at the same address
            Qd.copy_(to_dev(Q2))
        q = 2 if k >= 4 else 1
        check(out.call(B, idx, Qd, w.m, 3.5, precision), refs[(q, 3.5)], f"call {k}")
        # eager work in between: another radius into other buffers, and a
        # device op on torch's stream
        check(other.call(B, idx, Qd, w.m, 3.0, precision), refs[(q, 3.0)], f"other call {k}")
        Qd.mul_(1.0)


def test_replays_self_query_fp32(B):
    w = W.blobs3d(n=20_000, R=0.02)
    ref = oracle.brute_radius(w.P, w.P, w.R)
    say(f"graph replays: blobs3d self-query n={w.n} R={w.R} nnz={ref.col.size}")
    idx = B.Index(to_dev(w.P))
    out = FixedOut(w.n, ref.col.size + 1024)
    for k in range(4):
        check(out.call(B, idx, None, w.n, w.R, "auto", self_query=True), ref, f"self call {k}")


def test_replays_after_insert(B):
    w = W.gmm16(n=15_000, m=1_000, R=3.5)
    extra = W.gmm16(n=5_000, m=10, R=3.5, seed=5).P
    idx = B.Index(to_dev(w.P))
    Qd = to_dev(w.Q)
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    P2 = np.concatenate([w.P, extra])
    ref2 = oracle.brute_radius(P2, w.Q, w.R)
    say(f"graph replays around an insert: n={w.n}+{extra.shape[0]} m={w.m}")
    out = FixedOut(w.m, max(ref.col.size, ref2.col.size) + 1024)
    for k in range(3):
        check(out.call(B, idx, Qd, w.m, w.R, "auto"), ref, f"before insert {k}")
    idx.insert(to_dev(extra))
    for k in range(3):
        check(out.call(B, idx, Qd, w.m, w.R, "auto"), ref2, f"after insert {k}")
