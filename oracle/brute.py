"""O1: exhaustive fixed-radius search with the normative float64 distance.

Test infrastructure only (see the package docstring).

This is the "brute force 2" idea of Section 6.1 (SNN without an index and
without pruning) with the direct form of eq. (ip1) in place of gemv, so that
every decision is the normative one:

    S(p, q) = fl(...fl(fl(t_0^2) + fl(t_1^2)) ... + fl(t_{d-1}^2)),
    t_k = fl(p_k - q_k),

summed left to right exactly as the recursion of the rounding analysis in
Section 4 is written, with no fused multiply-add.  NumPy ufuncs round every
elementwise operation to float64 and never contract a multiply and an add,
so the loop over k below realises that recursion.  Neighbours are the i with
S(p_i, q) <= fl(R*R) (inclusive, Section 3.2).
"""

from __future__ import annotations

from typing import NamedTuple

import numpy as np


class Neighbors(NamedTuple):
    """CSR neighbour lists: row r holds col[row_ptr[r]:row_ptr[r+1]]."""

    row_ptr: np.ndarray  # int64, m+1
    col: np.ndarray  # int32, nnz, ascending within a row
    dist: np.ndarray  # float32, nnz, fl32(sqrt(S))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def normative_sqdist(P, q) -> np.ndarray:
    """S(p_i, q) for every row p_i of P (Section 4, eq. (ip1), left to right).

    P: (n, d) array, q: (d,) array; both promoted to float64 (exact).
    Returns float64 (n,).
    """
    P = _f64(P)
    q = _f64(q).reshape(-1)
    if P.ndim != 2 or P.shape[1] != q.shape[0]:
        raise ValueError("shape mismatch")
    s = np.zeros(P.shape[0], dtype=np.float64)
    for k in range(P.shape[1]):
        t = P[:, k] - q[k]
        s += t * t
    return s


def _block_sqdist(P: np.ndarray, Qb: np.ndarray) -> np.ndarray:
    """S for a block of queries: result[b, i] = S(P[i], Qb[b])."""
    s = np.zeros((Qb.shape[0], P.shape[0]), dtype=np.float64)
    t = np.empty_like(s)
    for k in range(P.shape[1]):
        np.subtract(P[None, :, k], Qb[:, k, None], out=t)
        np.multiply(t, t, out=t)
        s += t
    return s


def brute_radius(P, Q, R: float, max_block_elems: int = 1 << 22) -> Neighbors:
    """All i with S(P[i], Q[r]) <= fl(R*R), for every query row r.

    P: (n, d), Q: (m, d), R >= 0 finite.  Returns CSR with ascending ids per
    row and dist = fl32(sqrt(S)) computed in float64.
    """
    R = float(R)
    if not np.isfinite(R) or R < 0:
        raise ValueError("R must be finite and >= 0")
    return brute_sq_threshold(P, Q, R * R, max_block_elems)  # Python float multiply: one rounding


def brute_sq_threshold(P, Q, T2: float, max_block_elems: int = 1 << 22) -> Neighbors:
    """All i with S(P[i], Q[r]) <= T2 (a squared threshold given directly,
    e.g. the squared chord of an angle on unit vectors), dist = fl32(sqrt(S))."""
    P = _f64(P)
    Q = _f64(Q)
    if P.ndim != 2 or Q.ndim != 2 or P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must be 2-D with the same number of columns")
    R2 = float(T2)
    if not np.isfinite(R2) or R2 < 0:
        raise ValueError("the threshold must be finite and >= 0")
    n, m = P.shape[0], Q.shape[0]
    counts = np.zeros(m, dtype=np.int64)
    cols, dists = [], []
    blk = max(1, max_block_elems // max(n, 1))
    for b0 in range(0, m, blk):
        S = _block_sqdist(P, Q[b0 : b0 + blk])
        for r in range(S.shape[0]):
            idx = np.flatnonzero(S[r] <= R2)  # ascending
            counts[b0 + r] = idx.size
            cols.append(idx.astype(np.int32))
            dists.append(np.sqrt(S[r, idx]).astype(np.float32))
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    dist = np.concatenate(dists) if dists else np.zeros(0, np.float32)
    return Neighbors(row_ptr, col.astype(np.int32), dist.astype(np.float32))
