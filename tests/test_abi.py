"""The C-ABI library loads, exports every symbol include/snn.h declares, and
rejects bad arguments -- all without a GPU (no compute call is made)."""

import ctypes
import os
import re

import pytest

from paper_2212_07679_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("snn.h", "snn_testing.h")]


def declared_symbols():
    syms = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        syms.update(re.findall(r"\b(snn_[a-z0-9_]+)\s*\(", src))
    return sorted(syms)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("snn_index", "snn_query", "snn_query_self", "snn_index_free", "snn_last_error", "snn_debug_screen"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(declared_symbols()) <= set(B.SIGNATURES)


def test_version():
    assert B.lib().snn_version().decode().startswith("snn-mi355x")


def _dev():
    return B.snn_device(B.ALLOC_FN(), B.FREE_FN(), None, None, 0)


def test_index_argument_errors():
    L = B.lib()
    out = ctypes.c_void_p()
    dev = _dev()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: arguments are checked first
    assert L.snn_index(None, fake, 10, 2, 0, ctypes.byref(out)) == B.SNN_EINVAL
    assert L.snn_index(ctypes.byref(dev), None, 10, 2, 0, ctypes.byref(out)) == B.SNN_EINVAL
    assert L.snn_index(ctypes.byref(dev), fake, 0, 2, 0, ctypes.byref(out)) == B.SNN_EINVAL
    assert L.snn_index(ctypes.byref(dev), fake, 10, 0, 0, ctypes.byref(out)) == B.SNN_EINVAL
    assert L.snn_index(ctypes.byref(dev), fake, 10, 2000, 0, ctypes.byref(out)) == B.SNN_EINVAL
    assert L.snn_index(ctypes.byref(dev), fake, 10, 2, 7, ctypes.byref(out)) == B.SNN_EINVAL
    assert b"d must be" in L.snn_last_error() or b"dtype" in L.snn_last_error()


def test_query_argument_errors():
    L = B.lib()
    csr = B.snn_csr(0, 0, 0, 0, 0)
    assert L.snn_query(None, None, 1, 1.0, None, ctypes.byref(csr), None) == B.SNN_EINVAL
    assert L.snn_query_self(None, 1.0, None, ctypes.byref(csr), None) == B.SNN_EINVAL
    v = B.snn_index_view()
    assert L.snn_index_get_view(None, ctypes.byref(v)) == B.SNN_EINVAL
    L.snn_index_free(None)  # no-op


def test_batch_argument_errors():
    L = B.lib()
    dev = _dev()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: arguments are checked first
    csr = B.snn_csr(0, 0, 0, 0, 0)

    def inst(**kw):
        a = dict(X=fake.value, Q=None, n=100, m=0, d=3, R=0.1, out=ctypes.pointer(csr))
        a.update(kw)
        return (B.snn_instance * 1)(B.snn_instance(**a))

    h = ctypes.c_void_p()
    ok = inst()
    assert L.snn_batch_create(None, 0, ok, 1, None, ctypes.byref(h)) == B.SNN_EINVAL
    assert L.snn_batch_create(ctypes.byref(dev), 0, ok, 0, None, ctypes.byref(h)) == B.SNN_EINVAL
    assert L.snn_batch_create(ctypes.byref(dev), 0, None, 1, None, ctypes.byref(h)) == B.SNN_EINVAL
    assert L.snn_batch_create(ctypes.byref(dev), 7, ok, 1, None, ctypes.byref(h)) == B.SNN_EINVAL
    bad = [inst(X=None), inst(n=0), inst(d=0), inst(d=129), inst(R=-1.0), inst(R=float("nan")),
           inst(m=5), inst(Q=fake.value, m=-1), inst(out=None)]
    for b in bad:
        assert L.snn_batch_create(ctypes.byref(dev), 0, b, 1, None, ctypes.byref(h)) == B.SNN_EINVAL
        assert not h
    o = B.snn_batch_options(2, 0, 0, 0, None)
    assert L.snn_batch_create(ctypes.byref(dev), 0, ok, 1, ctypes.byref(o), ctypes.byref(h)) == B.SNN_EINVAL
    o = B.snn_batch_options(0, 100, 0, 0, None)
    assert L.snn_batch_create(ctypes.byref(dev), 0, ok, 1, ctypes.byref(o), ctypes.byref(h)) == B.SNN_EINVAL
    assert b"tile_c" in L.snn_last_error()
    st = B.snn_stats()
    assert L.snn_batch_run(None, 3, ctypes.byref(st)) == B.SNN_EINVAL
    inf = B.snn_batch_info_t()
    assert L.snn_batch_info(None, ctypes.byref(inf)) == B.SNN_EINVAL
    assert L.snn_query_batch(None, 0, ok, 1, None, None) == B.SNN_EINVAL
    L.snn_batch_free(None)  # no-op


def test_sort_argument_errors():
    L = B.lib()
    dev = _dev()
    fake = ctypes.c_void_p(0x1000)
    assert L.snn_sort_pairs_u32(None, fake, fake, 4, 0, 32) == B.SNN_EINVAL
    assert L.snn_sort_pairs_u32(ctypes.byref(dev), fake, fake, 4, 0, 33) == B.SNN_EINVAL
    assert L.snn_sort_pairs_u32(ctypes.byref(dev), fake, fake, 4, 8, 8) == B.SNN_EINVAL
    assert L.snn_sort_pairs_u32(ctypes.byref(dev), None, fake, 4, 0, 32) == B.SNN_EINVAL
    assert L.snn_sort_pairs_u32(ctypes.byref(dev), fake, fake, -1, 0, 32) == B.SNN_EINVAL


def test_dbscan_argument_errors():
    L = B.lib()
    dev = _dev()
    fake = ctypes.c_void_p(0x1000)
    k = ctypes.c_int64(0)
    assert L.snn_dbscan(None, 4, fake, fake, 5, fake, None, ctypes.byref(k)) == B.SNN_EINVAL
    assert L.snn_dbscan(ctypes.byref(dev), -1, fake, fake, 5, fake, None, ctypes.byref(k)) == B.SNN_EINVAL
    assert L.snn_dbscan(ctypes.byref(dev), 4, fake, fake, 0, fake, None, ctypes.byref(k)) == B.SNN_EINVAL
    assert L.snn_dbscan(ctypes.byref(dev), 4, None, fake, 5, fake, None, ctypes.byref(k)) == B.SNN_EINVAL
    assert L.snn_dbscan(ctypes.byref(dev), 4, fake, fake, 5, None, None, ctypes.byref(k)) == B.SNN_EINVAL
    assert L.snn_dbscan(ctypes.byref(dev), 2**31, fake, fake, 5, fake, None, ctypes.byref(k)) == B.SNN_EINVAL


def test_index_insert_argument_errors():
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.snn_index_insert(None, fake, 4) == B.SNN_EINVAL
    assert L.snn_index_insert(fake, fake, -1) == B.SNN_EINVAL
    assert L.snn_index_insert(fake, None, 4) == B.SNN_EINVAL


def test_dbscan_index_argument_errors():
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    k = ctypes.c_int64(0)
    assert L.snn_dbscan_index(None, 0.1, 5, None, fake, None, ctypes.byref(k), None) == B.SNN_EINVAL
    assert L.snn_dbscan_index(fake, 0.1, 0, None, fake, None, ctypes.byref(k), None) == B.SNN_EINVAL


@pytest.mark.skipif(os.path.exists("/dev/kfd"),
                    reason="a GPU may be present (the GPU driver is): the call below would then build an index "
                           "from a fake device pointer; the no-device path is only checked without a GPU driver")
def test_no_device_is_a_clean_error():
    L = B.lib()
    out = ctypes.c_void_p()
    dev = _dev()
    fake = ctypes.c_void_p(0x1000)
    assert L.snn_index(ctypes.byref(dev), fake, 10, 2, 0, ctypes.byref(out)) == B.SNN_EDEVICE
    assert b"device" in L.snn_last_error()


def test_debug_screen_argument_errors():
    L = B.lib()
    lay = B.snn_screen_layout()
    assert L.snn_debug_screen_layout(None, 1.0, None, ctypes.byref(lay)) == B.SNN_EINVAL
    assert L.snn_debug_screen(None, None, 1, 1.0, None, None, None, None, None, None, ctypes.byref(lay)) == B.SNN_EINVAL
