"""Allocator failure: when the caller's allocator returns NULL, every entry
point that allocates reports SNN_ENOMEM, frees everything it had allocated,
and leaves an existing index usable.  The failure is injected from the host
(the allocator callback); every kernel runs to its normal end."""

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


class FailingAllocator:
    """torch's caching allocator behind the snn_device callbacks, failing the
    allocation numbered fail_at (counted from 1) and every later one while
    armed; it tracks the live pointers it handed out."""

    def __init__(self, B, stream):
        self.live = {}
        self.count = 0
        self.fail_at = None
        dev, st = 0, stream

        def _alloc(_ctx, nbytes):
            self.count += 1
            if self.fail_at is not None and self.count >= self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
            self.live[p] = int(nbytes)
            return p

        def _free(_ctx, ptr):
            if ptr:
                assert ptr in self.live, "free of a pointer the allocator did not hand out"
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self._a = B.ALLOC_FN(_alloc)
        self._f = B.FREE_FN(_free)
        self.dev = B.snn_device(self._a, self._f, None, ctypes.c_void_p(st.cuda_stream), 0)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_index_build_fails_cleanly_at_every_allocation(B):
    w = W.gmm16(n=20_000, m=500, R=3.0)
    X = to_dev(w.P)
    stream = torch.cuda.Stream()
    al = FailingAllocator(B, stream)
    L = B.lib()
    h = ctypes.c_void_p()
    # allocations of a successful build
    torch.cuda.synchronize()
    assert L.snn_index(ctypes.byref(al.dev), ctypes.c_void_p(X.data_ptr()), w.n, w.d, B.SNN_F32, ctypes.byref(h)) == 0
    total = al.count
    L.snn_index_free(h)
    assert not al.live, "a successful build's free left allocations"
    say(f"index build: {total} allocations")
    for k in range(1, total + 1):
        al.count, al.fail_at = 0, k
        h = ctypes.c_void_p()
        st = L.snn_index(ctypes.byref(al.dev), ctypes.c_void_p(X.data_ptr()), w.n, w.d, B.SNN_F32, ctypes.byref(h))
        assert st == B.SNN_ENOMEM, f"allocation {k}: status {st}"
        assert not h, f"allocation {k}: index handle returned"
        assert not al.live, f"allocation {k}: {len(al.live)} allocations leaked"
        assert b"alloc" in L.snn_last_error().lower() or b"memory" in L.snn_last_error().lower()
    torch.cuda.synchronize()


def test_query_fails_cleanly_and_index_stays_usable(B):
    w = W.gmm16(n=20_000, m=2_000, R=3.5)
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    X, Q = to_dev(w.P), to_dev(w.Q)
    stream = torch.cuda.Stream()
    al = FailingAllocator(B, stream)
    L = B.lib()
    h = ctypes.c_void_p()
    torch.cuda.synchronize()
    assert L.snn_index(ctypes.byref(al.dev), ctypes.c_void_p(X.data_ptr()), w.n, w.d, B.SNN_F32, ctypes.byref(h)) == 0
    cap = ref.col.size + 1024
    row_ptr = torch.empty(w.m + 1, dtype=torch.int64, device="cuda:0")
    col = torch.empty(cap, dtype=torch.int32, device="cuda:0")
    dist = torch.empty(cap, dtype=torch.float32, device="cuda:0")

    def query(precision):
        csr = B.snn_csr(row_ptr.data_ptr(), col.data_ptr(), dist.data_ptr(), cap, 0)
        opts = B.snn_options(B.PRECISION[precision], 0, 0, 0, 0, 0)
        torch.cuda.synchronize()
        return L.snn_query(h, ctypes.c_void_p(Q.data_ptr()), w.m, float(w.R), ctypes.byref(opts), ctypes.byref(csr),
                           None), csr

    for precision in ("fp64", "auto", "mixed"):
        # the allocations of the query's first call (workspace, screen
        # operands) fail in turn; what succeeded before a failure stays with
        # the index (its workspace grows only) and is freed with it
        for k in range(1, 64):
            al.count, al.fail_at = 0, k
            st, _ = query(precision)
            if st == 0:
                break
            assert st == B.SNN_ENOMEM, f"{precision}, allocation {k}: status {st}"
        else:
            pytest.fail(f"{precision}: still failing after 63 allocations")
        al.fail_at = None
        st, csr = query(precision)
        assert st == 0
        nnz = int(csr.nnz)
        assert np.array_equal(row_ptr.cpu().numpy(), ref.row_ptr), precision
        assert np.array_equal(col[:nnz].cpu().numpy(), ref.col), precision
        say(f"query {precision}: {k - 1} allocation failures reported, then the call matched the oracle")
    L.snn_index_free(h)
    assert not al.live, f"{len(al.live)} allocations left after the index was freed"
