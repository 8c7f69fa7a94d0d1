"""ctypes binding of libsnn (include/snn.h): argument marshalling only.

Every step of index construction and querying runs in the library's HIP
kernels.  PyTorch provides device memory (its caching allocator, handed to
the library as the snn_device allocator) and the stream.  If libsnn.so is
missing, or the library reports an error, a ``SnnError`` is raised; there is
no fallback path.
"""

from __future__ import annotations

import contextlib
import ctypes
import os
import struct
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SNN_LIBRARY selects another build of the library (e.g. the sanitizer build
# the CPU ABI tests load); default: the in-tree libsnn.so
LIB_PATH = os.environ.get("SNN_LIBRARY") or os.path.join(_HERE, "libsnn.so")

SNN_OK, SNN_EINVAL, SNN_ENOMEM, SNN_EDEVICE, SNN_EOVERFLOW, SNN_ENOTSUP = 0, -1, -2, -3, -4, -5
SNN_F32, SNN_F64 = 0, 1
PRECISION = {"fp64": 0, "mixed": 1, "auto": 2, "fp32": 3, "fp16": 4}
PRECISION_NAMES = {v: k for k, v in PRECISION.items()}
METRIC = {"l2": 0, "l1": 1, "angular": 2, "cosine": 3}

STATUS_NAMES = {
    SNN_OK: "SNN_OK",
    SNN_EINVAL: "SNN_EINVAL",
    SNN_ENOMEM: "SNN_ENOMEM",
    SNN_EDEVICE: "SNN_EDEVICE",
    SNN_EOVERFLOW: "SNN_EOVERFLOW",
    SNN_ENOTSUP: "SNN_ENOTSUP",
}


class SnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class snn_device(ctypes.Structure):
    _fields_ = [
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("ctx", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("device", ctypes.c_int),
    ]


class snn_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("mixed_terms", ctypes.c_int),
        ("tile_q", ctypes.c_int),
        ("tile_c", ctypes.c_int),
        ("full_self_scan", ctypes.c_int),
        ("metric", ctypes.c_int),
    ]


class snn_csr(ctypes.Structure):
    _fields_ = [
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("dist", ctypes.c_void_p),
        ("nnz_cap", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
    ]


class snn_stats(ctypes.Structure):
    _fields_ = [
        ("pairs_window", ctypes.c_int64),
        ("pairs_executed", ctypes.c_int64),
        ("pairs_recheck", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("precision_used", ctypes.c_int32),
        ("terms_used", ctypes.c_int32),
        ("screen_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("flops_window", ctypes.c_double),
        ("stage_ms", ctypes.c_double * 5),
    ]

    def as_dict(self):
        # one unpack of the whole block (field-by-field ctypes reads cost
        # microseconds per call)
        v = struct.unpack_from(_STATS_FMT, self)
        d = dict(zip(_STATS_NAMES, v[:9]))
        d["stage_ms"] = list(v[9:])
        return d


_STATS_FMT = "<4q2i3d5d"
_STATS_NAMES = tuple(k for k, _ in snn_stats._fields_[:9])
assert struct.calcsize(_STATS_FMT) == ctypes.sizeof(snn_stats)


class snn_index_view(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int32),
        ("dtype", ctypes.c_int),
        ("mu", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("key", ctypes.c_void_p),
        ("perm", ctypes.c_void_p),
        ("max_norm", ctypes.c_double),
        ("key_eps", ctypes.c_double),
        ("power_iters", ctypes.c_int32),
    ]


class snn_instance(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("Q", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("d", ctypes.c_int32),
        ("R", ctypes.c_double),
        ("out", ctypes.POINTER(snn_csr)),
    ]


class snn_batch_options(ctypes.Structure):
    _fields_ = [
        ("mixed_terms", ctypes.c_int32),
        ("tile_c", ctypes.c_int32),
        ("tile_g", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
    ]


class snn_batch_info_t(ctypes.Structure):
    _fields_ = [
        ("tile_q", ctypes.c_int32),
        ("tile_c", ctypes.c_int32),
        ("tile_g", ctypes.c_int32),
        ("operand_k", ctypes.c_int32),
        ("graph_timed_screen", ctypes.c_int32),
        ("tuned_query_ms", ctypes.c_float),
        ("fp32_instances", ctypes.c_int32),
        ("fp32_k", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SNN_BATCH_INDEX, SNN_BATCH_QUERY = 1, 2


class snn_screen_layout(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("terms", ctypes.c_int32),
        ("ka", ctypes.c_int32),
        ("kb", ctypes.c_int32),
        ("chain", ctypes.c_int32),
        ("scale_exp", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

# symbol -> (restype, argtypes): every entry point declared in include/snn.h and
# include/snn_testing.h
SIGNATURES = {
    "snn_batch_create": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_int, ctypes.POINTER(snn_instance),
                                        ctypes.c_int32, ctypes.POINTER(snn_batch_options),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "snn_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(snn_stats)]),
    "snn_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(snn_batch_info_t)]),
    "snn_batch_free": (None, [ctypes.c_void_p]),
    "snn_query_batch": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_int, ctypes.POINTER(snn_instance),
                                       ctypes.c_int32, ctypes.POINTER(snn_batch_options),
                                       ctypes.POINTER(snn_stats)]),
    "snn_index": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "snn_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                 ctypes.POINTER(snn_options), ctypes.POINTER(snn_csr), ctypes.POINTER(snn_stats)]),
    "snn_query_self": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(snn_options),
                                      ctypes.POINTER(snn_csr), ctypes.POINTER(snn_stats)]),
    "snn_index_get_view": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(snn_index_view)]),
    "snn_index_free": (None, [ctypes.c_void_p]),
    "snn_index_insert": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "snn_sort_pairs_u32": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    "snn_sort_pairs_u32_noalloc": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    "snn_dbscan": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int64)]),
    "snn_dbscan_index": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(snn_options),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(snn_stats)]),
    "snn_normalize_rows": (ctypes.c_int, [ctypes.POINTER(snn_device), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int, ctypes.c_void_p]),
    "snn_debug_screen_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(snn_options),
                                               ctypes.POINTER(snn_screen_layout)]),
    "snn_debug_screen": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                        ctypes.POINTER(snn_options), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(snn_screen_layout)]),
    "snn_last_error": (ctypes.c_char_p, []),
    "snn_version": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libsnn.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SnnError(SNN_EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != SNN_OK:
        raise SnnError(status, lib().snn_last_error().decode())


_ALLOCATORS = {}


def _allocator(device: int, stream: Optional[torch.cuda.Stream] = None) -> "_TorchAllocator":
    """One allocator per (device, stream), shared by the indexes and plans on
    it (creating the ctypes callbacks costs tens of microseconds)."""
    st = stream if stream is not None else torch.cuda.current_stream(device)
    key = (device, st.cuda_stream)
    a = _ALLOCATORS.get(key)
    if a is None:
        a = _ALLOCATORS[key] = _TorchAllocator(device, st)
    return a


class _TorchAllocator:
    """snn_device backed by torch's caching allocator on one device/stream."""

    def __init__(self, device: int, stream: Optional[torch.cuda.Stream] = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        dev_id, st = device, self.stream

        def _alloc(_ctx, nbytes):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev_id, st)
            except Exception:  # out of memory -> NULL -> SNN_ENOMEM
                return None

        def _free(_ctx, ptr):
            if ptr:
                torch.cuda.caching_allocator_delete(ptr)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.dev = snn_device(self._alloc, self._free, None, ctypes.c_void_p(self.stream.cuda_stream), device)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return SNN_F32
    if t.dtype == torch.float64:
        return SNN_F64
    raise SnnError(SNN_EINVAL, f"unsupported dtype {t.dtype}")


def _device_tensor_from_ptr(ptr: int, count: int, dtype: torch.dtype, device: int) -> torch.Tensor:
    """Copy `count` elements at device address `ptr` into a new torch tensor."""
    out = torch.empty(count, dtype=dtype, device=f"cuda:{device}")
    if count:
        nbytes = count * out.element_size()
        hip = _hip()
        torch.cuda.synchronize(device)
        r = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes), 3)
        if r != 0:
            raise SnnError(SNN_EDEVICE, f"hipMemcpy failed ({r})")
    return out


_hiplib = None


def _hip():
    global _hiplib
    if _hiplib is None:
        _hiplib = ctypes.CDLL("libamdhip64.so")
        _hiplib.hipMemcpy.restype = ctypes.c_int
        _hiplib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hiplib


class Index:
    """An SNN index (Algorithm 1) over the rows of a device tensor X (n x d)."""

    def __init__(self, X: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
        if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dim() != 2:
            raise SnnError(SNN_EINVAL, "X must be a 2-D CUDA tensor")
        X = X.contiguous()
        self.device = X.device.index if X.device.index is not None else torch.cuda.current_device()
        self.dtype = X.dtype
        self.n, self.d = X.shape
        self._alloc = _allocator(self.device, stream)
        self._devobj = torch.device("cuda", self.device)
        self._h = ctypes.c_void_p()
        self._nnz_hint = 0
        self._opt_cache = {}
        self._csr_cache = {}
        _check(lib().snn_index(ctypes.byref(self._alloc.dev), ctypes.c_void_p(X.data_ptr()), self.n, self.d,
                               _dtype_code(X), ctypes.byref(self._h)))

    @property
    def stream(self) -> torch.cuda.Stream:
        return self._alloc.stream

    def close(self):
        if self._h:
            lib().snn_index_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _opts(self, precision: str, terms: int, tile_q: int, tile_c: int, full_self_scan: bool = False,
              metric: str = "l2") -> snn_options:
        # the library only reads the options: one object per distinct set
        key = (precision, terms, tile_q, tile_c, full_self_scan, metric)
        o = self._opt_cache.get(key)
        if o is None:
            o = self._opt_cache[key] = self._make_opts(*key)
        return o

    @staticmethod
    def _make_opts(precision: str, terms: int, tile_q: int, tile_c: int, full_self_scan: bool,
                   metric: str) -> snn_options:
        if precision not in PRECISION:
            raise SnnError(SNN_EINVAL, f"precision must be one of {sorted(PRECISION)}")
        if metric not in METRIC:
            raise SnnError(SNN_EINVAL, f"metric must be one of {sorted(METRIC)}")
        return snn_options(PRECISION[precision], int(terms), int(tile_q), int(tile_c), 1 if full_self_scan else 0,
                           METRIC[metric])

    def _run(self, Q: Optional[torch.Tensor], m: int, R: float, opts: snn_options, nnz_cap: Optional[int],
             want_stats: bool):
        dev = self._devobj
        # outputs are allocated for the index's stream (the caching allocator
        # ties a block to the stream current at allocation; the library may
        # still write them when the call returns)
        if torch.cuda.current_stream(self.device) == self.stream:
            ctx = contextlib.nullcontext()
        else:
            ctx = torch.cuda.stream(self.stream)
        with ctx:
            cap = int(nnz_cap) if nnz_cap is not None else max(self._nnz_hint, 4 * m, 1024)
            st = snn_stats() if want_stats else None
            stp = ctypes.byref(st) if want_stats else None
            L = lib()
            for _ in range(3):
                c1 = max(cap, 1)
                row_ptr = torch.empty(m + 1, dtype=torch.int64, device=dev)
                col = torch.empty(c1, dtype=torch.int32, device=dev)
                dist = torch.empty(c1, dtype=torch.float32, device=dev)
                csr = snn_csr(row_ptr.data_ptr(), col.data_ptr(), dist.data_ptr(), cap, 0)
                if Q is None:
                    status = L.snn_query_self(self._h, float(R), ctypes.byref(opts), ctypes.byref(csr), stp)
                else:
                    status = L.snn_query(self._h, Q.data_ptr(), m, float(R), ctypes.byref(opts), ctypes.byref(csr),
                                         stp)
                if status == SNN_EOVERFLOW and nnz_cap is None:
                    cap = int(csr.nnz)
                    continue
                _check(status)
                break
            nnz = int(csr.nnz)
            if nnz + (nnz >> 2) > self._nnz_hint:
                self._nnz_hint = nnz + (nnz >> 2)
            res = (row_ptr, col[:nnz], dist[:nnz])
            return (res + (st.as_dict(),)) if want_stats else res

    def query(self, Q: torch.Tensor, R: float, precision: str = "auto", terms: int = 0, tile_q: int = 0,
              tile_c: int = 0, nnz_cap: Optional[int] = None, stats: bool = False, metric: str = "l2"):
        """Algorithm 2 for the rows of Q (m x d, same dtype and device).
        ``metric``: "l2" (radius R), "l1" (Manhattan radius R), "angular"
        (R = angle in radians) or "cosine" (R = cosine distance); the last
        two expect unit rows (``normalize_rows``)."""
        if not isinstance(Q, torch.Tensor) or not Q.is_cuda or Q.dim() != 2 or Q.shape[1] != self.d:
            raise SnnError(SNN_EINVAL, "Q must be a CUDA tensor of shape (m, d)")
        if Q.dtype != self.dtype:
            raise SnnError(SNN_EINVAL, "Q must have the index dtype")
        Q = Q.contiguous()
        return self._run(Q, Q.shape[0], R, self._opts(precision, terms, tile_q, tile_c, metric=metric), nnz_cap, stats)

    def query_into(self, Q: Optional[torch.Tensor], R: float, row_ptr: torch.Tensor, col: torch.Tensor,
                   dist: torch.Tensor, precision: str = "auto", terms: int = 0, tile_q: int = 0, tile_c: int = 0,
                   stats: bool = False, metric: str = "l2", full_self_scan: bool = False):
        """Algorithm 2 into caller-owned output tensors (a serving loop's form:
        no allocation per call).  Q (m x d) or None for the all-points
        self-query; row_ptr: int64 with at least m + 1 entries; col / dist:
        int32 / float32 of one capacity.  Returns nnz (plus the stats dict);
        raises SnnError(SNN_EOVERFLOW) when the neighbours exceed the
        capacity (the message holds the count needed).  The tensors must be
        on the index's device; the library writes them on the index's stream
        (work on another stream that reads them must wait for it)."""
        m = self.n if Q is None else Q.shape[0]
        key = (row_ptr.data_ptr(), col.data_ptr(), dist.data_ptr(), col.numel(), dist.numel(), row_ptr.dtype,
               col.dtype, dist.dtype)
        csr = self._csr_cache.get(key)
        if csr is None:
            if (row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or dist.dtype != torch.float32
                    or dist.numel() != col.numel() or not (row_ptr.is_contiguous() and col.is_contiguous()
                                                            and dist.is_contiguous())):
                raise SnnError(SNN_EINVAL, "row_ptr / col / dist: contiguous int64 / int32 / float32, one capacity")
            if any(not t.is_cuda or t.device.index != self.device for t in (row_ptr, col, dist)):
                raise SnnError(SNN_EINVAL, "row_ptr / col / dist must be on the index's device")
            if len(self._csr_cache) > 16:
                self._csr_cache.clear()
            csr = self._csr_cache[key] = snn_csr(key[0], key[1], key[2], key[3], 0)
        if row_ptr.numel() < m + 1:
            raise SnnError(SNN_EINVAL, "row_ptr needs m + 1 entries")
        opts = self._opts(precision, terms, tile_q, tile_c, full_self_scan, metric)
        st = snn_stats() if stats else None
        if Q is None:
            status = lib().snn_query_self(self._h, float(R), ctypes.byref(opts), ctypes.byref(csr),
                                          ctypes.byref(st) if stats else None)
        else:
            if not Q.is_cuda or Q.dim() != 2 or Q.shape[1] != self.d or Q.dtype != self.dtype or not Q.is_contiguous():
                raise SnnError(SNN_EINVAL, "Q must be a contiguous CUDA tensor of shape (m, d) and the index dtype")
            status = lib().snn_query(self._h, Q.data_ptr(), m, float(R), ctypes.byref(opts), ctypes.byref(csr),
                                     ctypes.byref(st) if stats else None)
        _check(status)
        nnz = csr.nnz
        return (nnz, st.as_dict()) if stats else nnz

    def query_self(self, R: float, precision: str = "auto", terms: int = 0, tile_q: int = 0, tile_c: int = 0,
                   nnz_cap: Optional[int] = None, stats: bool = False, full_self_scan: bool = False,
                   metric: str = "l2"):
        """Every data row as a query (rows in original data order).  Each
        unordered pair is scanned once unless ``full_self_scan``."""
        return self._run(None, self.n, R, self._opts(precision, terms, tile_q, tile_c, full_self_scan, metric),
                         nnz_cap, stats)

    def insert(self, X: torch.Tensor) -> None:
        """Append the rows of X (k x d, the index dtype) as points n .. n+k-1
        (streaming inserts: the index's centre and direction are kept)."""
        if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dim() != 2 or X.shape[1] != self.d:
            raise SnnError(SNN_EINVAL, "X must be a CUDA tensor of shape (k, d)")
        if X.dtype != self.dtype:
            raise SnnError(SNN_EINVAL, "X must have the index dtype")
        X = X.contiguous()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            _check(lib().snn_index_insert(self._h, ctypes.c_void_p(X.data_ptr()), X.shape[0]))
        self.n += X.shape[0]

    def dbscan(self, eps: float, min_samples: int = 5, precision: str = "auto", stats: bool = False,
               full_self_scan: bool = False, metric: str = "l2"):
        """DBSCAN (Section 6.4) of the indexed points with eps-neighbourhoods
        of this index's self-query, clustered on the device without
        assembling the neighbour lists.  Returns ``(labels, core, nclusters)``
        (plus the stats dict): int32 labels in the original point order (-1
        noise, clusters numbered by smallest core id), a bool core mask."""
        opts = self._opts(precision, 0, 0, 0, full_self_scan, metric)
        dev = f"cuda:{self.device}"
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            labels = torch.empty(max(self.n, 1), dtype=torch.int32, device=dev)
            core = torch.empty(max(self.n, 1), dtype=torch.uint8, device=dev)
            k = ctypes.c_int64(0)
            st = snn_stats()
            _check(lib().snn_dbscan_index(self._h, float(eps), int(min_samples), ctypes.byref(opts),
                                          ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(core.data_ptr()),
                                          ctypes.byref(k), ctypes.byref(st)))
            core = core[:self.n].bool()
        res = (labels[:self.n], core, int(k.value))
        return (res + (st.as_dict(),)) if stats else res

    def screen_values(self, Q: torch.Tensor, R: float, precision: str = "auto", terms: int = 0) -> dict:
        """Test support (include/snn_testing.h): every (query, candidate)
        pair's screen value D, the candidates' H, the queries' start values
        C and both operand row sets of the screen a query would run."""
        if not isinstance(Q, torch.Tensor) or not Q.is_cuda or Q.dim() != 2 or Q.shape[1] != self.d:
            raise SnnError(SNN_EINVAL, "Q must be a CUDA tensor of shape (m, d)")
        if Q.dtype != self.dtype:
            raise SnnError(SNN_EINVAL, "Q must have the index dtype")
        Q = Q.contiguous()
        opts = self._opts(precision, terms, 0, 0)
        lay = snn_screen_layout()
        _check(lib().snn_debug_screen_layout(self._h, float(R), ctypes.byref(opts), ctypes.byref(lay)))
        m, n = Q.shape[0], self.n
        dev = f"cuda:{self.device}"
        vt = torch.float32 if lay.precision == PRECISION["fp32"] else torch.int16
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            D = torch.empty((m, n), dtype=torch.float32, device=dev)
            H = torch.empty(n, dtype=torch.float32, device=dev)
            C = torch.empty(m, dtype=torch.float32, device=dev)
            A = torch.empty((m, lay.ka), dtype=vt, device=dev)
            Bm = torch.empty((n, lay.kb), dtype=vt, device=dev)
            _check(lib().snn_debug_screen(self._h, ctypes.c_void_p(Q.data_ptr()), m, float(R), ctypes.byref(opts),
                                          ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(H.data_ptr()),
                                          ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(A.data_ptr()),
                                          ctypes.c_void_p(Bm.data_ptr()), ctypes.byref(lay)))
        return {"layout": lay.as_dict(), "D": D, "H": H, "C": C, "A": A, "B": Bm}

    def view(self) -> dict:
        """Index internals copied into new tensors (for checks)."""
        v = snn_index_view()
        _check(lib().snn_index_get_view(self._h, ctypes.byref(v)))
        torch.cuda.synchronize(self.device)
        return {
            "n": v.n,
            "d": v.d,
            "mu": _device_tensor_from_ptr(v.mu, v.d, torch.float64, self.device),
            "v": _device_tensor_from_ptr(v.v, v.d, torch.float64, self.device),
            "key": _device_tensor_from_ptr(v.key, v.n, torch.float64, self.device),
            "perm": _device_tensor_from_ptr(v.perm, v.n, torch.int32, self.device),
            "max_norm": v.max_norm,
            "key_eps": v.key_eps,
            "power_iters": v.power_iters,
        }


def sort_pairs_u32(keys: torch.Tensor, vals: torch.Tensor, begin_bit: int = 0, end_bit: int = 32) -> None:
    """Stable LSD radix sort of (keys, vals) in place (uint32 data in int32 tensors)."""
    if keys.shape != vals.shape or keys.dim() != 1 or not keys.is_cuda or not vals.is_cuda:
        raise SnnError(SNN_EINVAL, "keys and vals must be 1-D CUDA tensors of equal length")
    if keys.dtype not in (torch.int32, torch.uint32) or vals.dtype not in (torch.int32, torch.uint32):
        raise SnnError(SNN_EINVAL, "keys and vals must be 32-bit")
    if not keys.is_contiguous() or not vals.is_contiguous():
        raise SnnError(SNN_EINVAL, "keys and vals must be contiguous")
    device = keys.device.index
    alloc = _allocator(device)
    _check(lib().snn_sort_pairs_u32(ctypes.byref(alloc.dev), ctypes.c_void_p(keys.data_ptr()),
                                    ctypes.c_void_p(vals.data_ptr()), keys.numel(), begin_bit, end_bit))


def sort_pairs_u32_noalloc(keys: torch.Tensor, vals: torch.Tensor, begin_bit: int = 0, end_bit: int = 32,
                           stream: Optional[torch.cuda.Stream] = None) -> None:
    """The same sort through the allocation-free entry point (static device
    workspace, at most 2^21 pairs); enqueued on ``stream`` (default: the
    current stream) without waiting."""
    if keys.shape != vals.shape or keys.dim() != 1 or not keys.is_cuda or not vals.is_cuda:
        raise SnnError(SNN_EINVAL, "keys and vals must be 1-D CUDA tensors of equal length")
    if keys.dtype not in (torch.int32, torch.uint32) or vals.dtype not in (torch.int32, torch.uint32):
        raise SnnError(SNN_EINVAL, "keys and vals must be 32-bit")
    if not keys.is_contiguous() or not vals.is_contiguous():
        raise SnnError(SNN_EINVAL, "keys and vals must be contiguous")
    device = keys.device.index
    st = stream if stream is not None else torch.cuda.current_stream(device)
    dev = snn_device(ALLOC_FN(), FREE_FN(), None, ctypes.c_void_p(st.cuda_stream), device)
    _check(lib().snn_sort_pairs_u32_noalloc(ctypes.byref(dev), ctypes.c_void_p(keys.data_ptr()),
                                            ctypes.c_void_p(vals.data_ptr()), keys.numel(), begin_bit, end_bit))


def normalize_rows(X: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Rows scaled to unit Euclidean norm (float64 rule, one rounding to the
    dtype), for angular and cosine neighbours; ``out`` may be ``X``."""
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dim() != 2:
        raise SnnError(SNN_EINVAL, "X must be a 2-D CUDA tensor")
    X = X.contiguous()
    if out is None:
        out = torch.empty_like(X)
    if out.shape != X.shape or out.dtype != X.dtype or not out.is_contiguous() or out.device != X.device:
        raise SnnError(SNN_EINVAL, "out must be a contiguous tensor like X")
    device = X.device.index if X.device.index is not None else torch.cuda.current_device()
    alloc = _allocator(device)
    _check(lib().snn_normalize_rows(ctypes.byref(alloc.dev), ctypes.c_void_p(X.data_ptr()), X.shape[0], X.shape[1],
                                    _dtype_code(X), ctypes.c_void_p(out.data_ptr())))
    return out


def dbscan_csr(row_ptr: torch.Tensor, col: torch.Tensor, min_samples: int = 5,
               stream: Optional[torch.cuda.Stream] = None):
    """DBSCAN labels from all-points self-query lists (Section 6.4).

    row_ptr (n+1, int64) and col (int32) are CUDA tensors as returned by
    ``Index.query_self``; the work runs on ``stream`` (default: the current
    stream), which must be ordered after the producer of the lists.  Returns ``(labels, core, nclusters)``: int32 labels
    (-1 noise, clusters numbered by smallest core id), a bool core mask and
    the cluster count."""
    for t, dt, name in ((row_ptr, torch.int64, "row_ptr"), (col, torch.int32, "col")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dim() != 1 or t.dtype != dt:
            raise SnnError(SNN_EINVAL, f"{name} must be a 1-D CUDA {dt} tensor")
    if row_ptr.numel() < 1:
        raise SnnError(SNN_EINVAL, "row_ptr must hold n + 1 entries")
    row_ptr = row_ptr.contiguous()
    col = col.contiguous()
    n = row_ptr.numel() - 1
    device = row_ptr.device.index if row_ptr.device.index is not None else torch.cuda.current_device()
    alloc = _allocator(device, stream)
    with torch.cuda.device(device), torch.cuda.stream(alloc.stream):
        labels = torch.empty(max(n, 1), dtype=torch.int32, device=f"cuda:{device}")
        core = torch.empty(max(n, 1), dtype=torch.uint8, device=f"cuda:{device}")
        k = ctypes.c_int64(0)
        _check(lib().snn_dbscan(ctypes.byref(alloc.dev), n, ctypes.c_void_p(row_ptr.data_ptr()),
                                ctypes.c_void_p(col.data_ptr()), int(min_samples), ctypes.c_void_p(labels.data_ptr()),
                                ctypes.c_void_p(core.data_ptr()), ctypes.byref(k)))
        core = core[:n].bool()
    return labels[:n], core, int(k.value)


def dbscan(X: torch.Tensor, eps: float, min_samples: int = 5, precision: str = "auto"):
    """DBSCAN of the rows of X: SNN index, then ``Index.dbscan`` (the
    self-query's accepted pairs clustered on the device).  Returns
    ``(labels, core, nclusters)``."""
    idx = Index(X)
    try:
        return idx.dbscan(eps, min_samples, precision=precision)
    finally:
        idx.close()


class Batch:
    """A plan of many independent instances (the batching form).

    ``instances`` is a list of ``(X, Q, R)`` with X (n x d) and Q (m x d, or
    None for an all-points self-query) CUDA tensors of one dtype.  Creating
    the plan runs both passes once; ``run()`` launches the captured graph
    again (after the data in X / Q changed, or to time it) and returns one
    ``(row_ptr, col, dist)`` per instance.  The tensors must stay alive and
    keep their shapes while the plan exists.
    """

    def __init__(self, instances, terms: int = 0, tile_c: int = 0, tile_g: int = 0, autotune: bool = False,
                 tune_cache: Optional[str] = None, nnz_caps=None, stream: Optional[torch.cuda.Stream] = None):
        if not instances:
            raise SnnError(SNN_EINVAL, "no instances")
        X0 = instances[0][0]
        if not isinstance(X0, torch.Tensor) or not X0.is_cuda:
            raise SnnError(SNN_EINVAL, "X must be CUDA tensors")
        self.dtype = X0.dtype
        self.device = X0.device.index if X0.device.index is not None else torch.cuda.current_device()
        self._alloc = _allocator(self.device, stream)
        self._keep = []
        self.count = len(instances)
        self._csr = (snn_csr * self.count)()
        self._inst = (snn_instance * self.count)()
        self._out = []
        dev = f"cuda:{self.device}"
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            for i, (X, Q, R) in enumerate(instances):
                if not isinstance(X, torch.Tensor) or X.dim() != 2 or X.dtype != self.dtype or not X.is_cuda:
                    raise SnnError(SNN_EINVAL, f"instance {i}: X must be a 2-D CUDA tensor of the batch dtype")
                if not X.is_contiguous():
                    raise SnnError(SNN_EINVAL, f"instance {i}: X must be contiguous")
                n, d = X.shape
                if Q is not None:
                    if (not isinstance(Q, torch.Tensor) or Q.dim() != 2 or Q.shape[1] != d or Q.dtype != self.dtype
                            or not Q.is_cuda or not Q.is_contiguous()):
                        raise SnnError(SNN_EINVAL, f"instance {i}: Q must be a contiguous (m, d) CUDA tensor")
                    m = Q.shape[0]
                else:
                    m = n
                cap = int(nnz_caps[i]) if nnz_caps is not None else max(32 * m, 1024)
                row_ptr = torch.empty(m + 1, dtype=torch.int64, device=dev)
                col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
                dist = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
                self._out.append([row_ptr, col, dist])
                self._csr[i] = snn_csr(row_ptr.data_ptr(), col.data_ptr(), dist.data_ptr(), cap, 0)
                # Q NULL means a self-query when m = n and no queries when m = 0
                qp = Q.data_ptr() if (Q is not None and m > 0) else None
                self._inst[i] = snn_instance(X.data_ptr(), qp, n, m, d, float(R), ctypes.pointer(self._csr[i]))
                self._keep.append((X, Q))
            self._cache = tune_cache.encode() if tune_cache else None
            opts = snn_batch_options(int(terms), int(tile_c), int(tile_g), 1 if autotune else 0, self._cache)
            self._h = ctypes.c_void_p()
            _check(lib().snn_batch_create(ctypes.byref(self._alloc.dev), _dtype_code(X0), self._inst, self.count,
                                          ctypes.byref(opts), ctypes.byref(self._h)))

    @property
    def stream(self) -> torch.cuda.Stream:
        return self._alloc.stream

    def info(self) -> dict:
        inf = snn_batch_info_t()
        _check(lib().snn_batch_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def run(self, index: bool = True, query: bool = True, stats: bool = False, views: bool = True):
        """Launches the pass(es) and waits.  Returns one (row_ptr, col, dist)
        per instance (views of the output buffers cut at nnz), or with
        ``views=False`` only the nnz of each instance (the lists are the first
        nnz entries of ``buffers()[i]``; no tensor is made per call)."""
        what = (SNN_BATCH_INDEX if index else 0) | (SNN_BATCH_QUERY if query else 0)
        dev = f"cuda:{self.device}"
        st = snn_stats()
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            for _ in range(3):
                status = lib().snn_batch_run(self._h, what, ctypes.byref(st))
                if status != SNN_EOVERFLOW:
                    _check(status)
                    break
                # grow the outputs that overflowed; the index pass is done
                for i in range(self.count):
                    c = self._csr[i]
                    if c.nnz > c.nnz_cap:
                        cap = int(c.nnz + c.nnz // 4 + 16)
                        col = torch.empty(cap, dtype=torch.int32, device=dev)
                        dist = torch.empty(cap, dtype=torch.float32, device=dev)
                        self._out[i][1:] = [col, dist]
                        c.col, c.dist, c.nnz_cap = col.data_ptr(), dist.data_ptr(), cap
                what = SNN_BATCH_QUERY
            else:
                _check(status)
        if not query:
            return st.as_dict() if stats else None
        if views:
            res = [(o[0], o[1][: int(self._csr[i].nnz)], o[2][: int(self._csr[i].nnz)]) for i, o in enumerate(self._out)]
        else:
            res = [int(c.nnz) for c in self._csr]
        return (res, st.as_dict()) if stats else res

    def buffers(self):
        """The output buffers (row_ptr, col, dist) of every instance."""
        return [tuple(o) for o in self._out]

    def close(self):
        if getattr(self, "_h", None):
            lib().snn_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
