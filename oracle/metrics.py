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
  right, of |fl(p_k - q_k)|; distances fl32(M);
* angular (angle a in radians) and cosine (distance c) on unit rows: the
  normative S compared with the squared chord T = fl(2 - 2 cos(a)) (Python's
  float cosine) or T = fl(2c); distances fl32(2 asin(min(1, sqrt(S)/2))) (the
  angle) or fl32(S/2) (the cosine distance), evaluated in float64.
"""

from __future__ import annotations

import math

import numpy as np

from .brute import Neighbors, brute_sq_threshold
from .snn import query as snn_query


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


def angular_threshold(alpha: float) -> float:
    """Squared chord of the angle alpha on unit vectors: fl(2 - 2 cos(alpha))."""
    alpha = float(alpha)
    if not (0.0 <= alpha <= math.pi):
        raise ValueError("the angle must be in [0, pi]")
    return 2.0 - 2.0 * math.cos(alpha)


def cosine_threshold(c: float) -> float:
    """Squared chord of cosine distance c on unit vectors: fl(2c)."""
    c = float(c)
    if not np.isfinite(c) or c < 0:
        raise ValueError("the cosine distance must be finite and >= 0")
    return 2.0 * c


def _angle_dist(S):
    return (2.0 * np.arcsin(np.minimum(1.0, 0.5 * np.sqrt(S)))).astype(np.float32)


def _cosine_dist(S):
    return (0.5 * S).astype(np.float32)


def _search_sq(P, Q, T2, dist_of):
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    nb = brute_sq_threshold(P, Q, T2)
    S = np.empty(nb.col.size)
    for r in range(Q.shape[0]):
        a, b = nb.row_ptr[r], nb.row_ptr[r + 1]
        if b > a:
            t = P[nb.col[a:b]] - Q[r]
            s = np.zeros(b - a)
            for k in range(P.shape[1]):
                s = s + t[:, k] * t[:, k]
            S[a:b] = s
    return nb._replace(dist=dist_of(S))


def brute_angular(P, Q, alpha: float) -> Neighbors:
    """Exhaustive angular search of unit rows: S <= fl(2 - 2 cos(alpha))."""
    return _search_sq(P, Q, angular_threshold(alpha), _angle_dist)


def brute_cosine(P, Q, c: float) -> Neighbors:
    """Exhaustive cosine-distance search of unit rows: S <= fl(2c)."""
    return _search_sq(P, Q, cosine_threshold(c), _cosine_dist)


def snn_angular(index, Q, alpha: float):
    """Algorithm 2 (the CPU SNN) for an angular search of unit rows: the
    window is cut with the chord radius rounded up, decisions use the squared
    chord itself.  Returns (Neighbors with angles, stats)."""
    T2 = angular_threshold(alpha)
    R = float(np.nextafter(math.sqrt(T2), np.inf))
    nb, st = snn_query(index, Q, R, R2=T2)
    # the angle from the returned fl32(sqrt(S)): within a few fp32 ulps of the
    # angle of S itself, which the 1e-5 relative distance tolerance allows
    S = nb.dist.astype(np.float64) ** 2
    return nb._replace(dist=_angle_dist(S)), st
