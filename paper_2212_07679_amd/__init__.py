"""MI355X-native SNN query phase (exact fixed-radius near-neighbour search).

The compute path lives in ``libsnn.so`` (hand-written HIP kernels for gfx950
behind a C ABI, declared in ``include/snn.h``); ``binding`` is a thin ctypes
layer over it.  Importing this package loads nothing: the library is opened
on first use and a missing library is an error, never a fallback.
"""

__all__ = ["binding", "workloads"]
