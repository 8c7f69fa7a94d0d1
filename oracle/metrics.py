"""Other distances of Section 2 on top of the Euclidean search.

Test infrastructure only (see the package docstring).

Section 2 notes that the method serves further distances:

* cosine and angular distance on normalised vectors: for unit u, v the
  cosine distance is ||u - v||^2 / 2 and the angle is at most a iff
  ||u - v||^2 <= 2 - 2 cos(a), so both are Euclidean radius searches of the
  normalised rows, with R = sqrt(2c) or sqrt(2 - 2 cos(a));
* the Manhattan distance: the 2-norm never exceeds the 1-norm, so every
  Manhattan neighbour within R is a Euclidean neighbour within R and the
  same pruning applies.

Result definitions (the readings the GPU path follows):

* normalisation: y_k = fl(x_k / sqrt(s)), s the float64 sum of x_k^2 left to
  right, the quotient rounded once to the row dtype (float64 promotion of
  the inputs is exact);
* Manhattan: N1(q) = { i : M(p_i, q) <= R } with M the float64 sum, left to
  right, of |fl(p_k - q_k)|; distances fl32(M).
"""

from __future__ import annotations

import numpy as np

from .brute import Neighbors


def normalize_rows(X) -> np.ndarray:
    """Rows of X scaled to unit norm by the rule above, in X's dtype.

    Raises ValueError for a zero or non-finite row.
    """
    X = np.asarray(X)
    dt = X.dtype if X.dtype in (np.float32, np.float64) else np.float64
    X64 = X.astype(np.float64)
    s = np.zeros(X64.shape[0])
    for k in range(X64.shape[1]):
        s = s + X64[:, k] * X64[:, k]
    nrm = np.sqrt(s)
    if not np.all(np.isfinite(nrm)) or np.any(nrm == 0.0):
        raise ValueError("zero or non-finite row")
    return (X64 / nrm[:, None]).astype(dt)


def manhattan(P, q) -> np.ndarray:
    """M(p_i, q) for every row of P: float64, left to right over coordinates."""
    P = np.ascontiguousarray(np.asarray(P), dtype=np.float64)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    if P.ndim != 2 or P.shape[1] != q.shape[0]:
        raise ValueError("shape mismatch")
    s = np.zeros(P.shape[0])
    for k in range(P.shape[1]):
        s = s + np.abs(P[:, k] - q[k])
    return s


def brute_l1(P, Q, R: float) -> Neighbors:
    """Exhaustive Manhattan radius search (inclusive, ids ascending)."""
    P = np.asarray(P)
    Q = np.asarray(Q)
    if Q.ndim == 1:
        Q = Q.reshape(1, -1)
    if R < 0 or not np.isfinite(R):
        raise ValueError("R must be finite and >= 0")
    rows, cols, dists = [0], [], []
    for j in range(Q.shape[0]):
        m = manhattan(P, Q[j])
        idx = np.flatnonzero(m <= R)
        cols.append(idx.astype(np.int32))
        dists.append(m[idx].astype(np.float32))
        rows.append(rows[-1] + idx.size)
    return Neighbors(np.asarray(rows, dtype=np.int64),
                     np.concatenate(cols) if cols else np.zeros(0, np.int32),
                     np.concatenate(dists) if dists else np.zeros(0, np.float32))
