"""The allocation-free entry point snn_sort_pairs_u32_noalloc (static device
workspace) against the allocating snn_sort_pairs_u32, called through the C
ABI: two calls in a row, the second on a smaller input, each compared bit
for bit with the allocating sort of the same input (and with numpy's stable
argsort), plus the size limit."""

import ctypes
import sys

import numpy as np
import pytest

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


def keys_vals(n, seed):
    g = np.random.default_rng([2212, 7679, 31, seed])
    k = g.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    k[: n // 3] &= np.uint32(0xFF0FFFFF)  # many equal digits: stability matters
    v = np.arange(n, dtype=np.uint32)
    return k, v


def run_noalloc(B, keys, vals, begin, end):
    L = B.lib()
    st = torch.cuda.current_stream()
    dev = B.snn_device(B.ALLOC_FN(), B.FREE_FN(), None, ctypes.c_void_p(st.cuda_stream), keys.device.index)
    rc = L.snn_sort_pairs_u32_noalloc(ctypes.byref(dev), ctypes.c_void_p(keys.data_ptr()),
                                      ctypes.c_void_p(vals.data_ptr()), keys.numel(), begin, end)
    return rc


@pytest.mark.parametrize("bits", [(0, 32), (8, 28)])
def test_noalloc_matches_allocating_sort(B, bits):
    begin, end = bits
    for call, n in enumerate((1_900_003, 70_001)):  # second call smaller: stale workspace contents must not matter
        say(f"noalloc sort call {call}: n={n} bits={bits}")
        k, v = keys_vals(n, 10 * call + begin)
        ka = torch.from_numpy(k.view(np.int32)).cuda()
        va = torch.from_numpy(v.view(np.int32)).cuda()
        kb, vb = ka.clone(), va.clone()
        assert run_noalloc(B, ka, va, begin, end) == B.SNN_OK, B.lib().snn_last_error()
        B.sort_pairs_u32(kb, vb, begin, end)
        torch.cuda.synchronize()
        assert torch.equal(ka, kb) and torch.equal(va, vb), f"call {call}: differs from the allocating sort"
        mask = np.uint32(((1 << (end - begin)) - 1) << begin) if end - begin < 32 else np.uint32(0xFFFFFFFF)
        order = np.argsort(k & mask, kind="stable")
        assert np.array_equal(va.cpu().numpy().view(np.uint32), v[order])


def test_noalloc_limits(B):
    say("noalloc sort limits")
    n = (1 << 21) + 1
    k = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    v = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    assert run_noalloc(B, k, v, 0, 32) == B.SNN_EINVAL
    assert b"exceeds the static scratch" in B.lib().snn_last_error()
    assert run_noalloc(B, k[:10], v[:10], 0, 33) == B.SNN_EINVAL
    # the largest size it takes, and empty / single inputs
    kk, vv = keys_vals(1 << 21, 5)
    ka = torch.from_numpy(kk.view(np.int32)).cuda()
    va = torch.from_numpy(vv.view(np.int32)).cuda()
    assert run_noalloc(B, ka, va, 0, 32) == B.SNN_OK
    torch.cuda.synchronize()
    assert np.array_equal(va.cpu().numpy().view(np.uint32), vv[np.argsort(kk, kind="stable")])
    assert run_noalloc(B, ka[:0], va[:0], 0, 32) == B.SNN_OK
    assert run_noalloc(B, ka[:1], va[:1], 0, 32) == B.SNN_OK
    torch.cuda.synchronize()
