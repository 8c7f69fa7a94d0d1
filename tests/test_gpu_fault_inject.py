"""Injected HIP failures (SNN_FAULT_INJECT=n: the n-th checked HIP result of
an entry point's call reads as a failure).  For every n until the call
succeeds, the index build and the query must return SNN_EDEVICE with the
injected message, free what they allocated, and leave an existing index
usable: the next call without injection equals the oracle.  The failures
are host-side only; every kernel that was launched runs to its normal end."""

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


class CountingAllocator:
    """torch's caching allocator behind the snn_device callbacks, tracking the
    live pointers it handed out."""

    def __init__(self, B, stream):
        self.live = {}
        dev, st = 0, stream

        def _alloc(_ctx, nbytes):
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


def test_index_build_fails_cleanly_at_every_check(B, monkeypatch):
    w = W.gmm16(n=20_000, m=500, R=3.0)
    X = to_dev(w.P)
    stream = torch.cuda.Stream()
    al = CountingAllocator(B, stream)
    L = B.lib()
    torch.cuda.synchronize()
    n_fail = 0
    for k in range(1, 400):
        monkeypatch.setenv("SNN_FAULT_INJECT", str(k))
        h = ctypes.c_void_p()
        st = L.snn_index(ctypes.byref(al.dev), ctypes.c_void_p(X.data_ptr()), w.n, w.d, B.SNN_F32, ctypes.byref(h))
        monkeypatch.delenv("SNN_FAULT_INJECT")
        if st == 0:
            L.snn_index_free(h)
            break
        assert st == B.SNN_EDEVICE, (k, st)
        assert b"injected" in L.snn_last_error(), L.snn_last_error()
        assert not h.value
        stream.synchronize()
        assert not al.live, f"check {k}: the failed build left {len(al.live)} allocations"
        n_fail += 1
    else:
        pytest.fail("the build never succeeded")
    say(f"index build: {n_fail} injected failures, each clean")
    assert n_fail > 10
    assert not al.live


@pytest.mark.parametrize("precision", ["auto", "fp64"])
def test_query_fails_cleanly_at_every_check(B, monkeypatch, precision):
    w = W.gmm16(n=20_000, m=500, R=3.0)
    ref = oracle.brute_radius(w.P, w.Q, w.R)
    X, Q = to_dev(w.P), to_dev(w.Q)
    stream = torch.cuda.Stream()
    al = CountingAllocator(B, stream)
    L = B.lib()
    torch.cuda.synchronize()
    h = ctypes.c_void_p()
    assert L.snn_index(ctypes.byref(al.dev), ctypes.c_void_p(X.data_ptr()), w.n, w.d, B.SNN_F32, ctypes.byref(h)) == 0
    cap = ref.col.size + 256
    row_ptr = torch.empty(w.m + 1, dtype=torch.int64, device="cuda:0")
    col = torch.empty(cap, dtype=torch.int32, device="cuda:0")
    dist = torch.empty(cap, dtype=torch.float32, device="cuda:0")
    opts = B.snn_options(B.PRECISION[precision], 0, 0, 0, 0, 0)

    def query(stats):
        csr = B.snn_csr(row_ptr.data_ptr(), col.data_ptr(), dist.data_ptr(), cap, 0)
        s = B.snn_stats()
        r = L.snn_query(h, ctypes.c_void_p(Q.data_ptr()), w.m, float(w.R), ctypes.byref(opts), ctypes.byref(csr),
                        ctypes.byref(s) if stats else None)
        return r, csr

    def check_clean(what):
        r, csr = query(True)
        assert r == 0, (what, r, L.snn_last_error())
        stream.synchronize()
        assert np.array_equal(row_ptr.cpu().numpy(), ref.row_ptr), what
        assert np.array_equal(col[: csr.nnz].cpu().numpy(), ref.col), what

    check_clean("before")
    n_fail = 0
    for k in range(1, 400):
        monkeypatch.setenv("SNN_FAULT_INJECT", str(k))
        r, _ = query(True)
        monkeypatch.delenv("SNN_FAULT_INJECT")
        if r == 0:
            break
        assert r == B.SNN_EDEVICE, (k, r)
        assert b"injected" in L.snn_last_error(), L.snn_last_error()
        n_fail += 1
        check_clean(f"after injected failure {k}")
    else:
        pytest.fail("the query never succeeded")
    say(f"query ({precision}): {n_fail} injected failures, each followed by a correct query")
    assert n_fail > 3
    check_clean("after")
    L.snn_index_free(h)
    stream.synchronize()
    assert not al.live, f"{len(al.live)} allocations left after the index was freed"
