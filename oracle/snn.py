"""O2: SNN on the CPU -- Algorithm 1 (index) and Algorithm 2 (query), Section 3.

Test infrastructure only (see the package docstring).

Index (Algorithm 1, Section 3.1): centre by the empirical mean, take the
first principal component v1 of the centred matrix X (thin SVD, eq. (svd)),
score alpha_i = x_i^T v1, sort the rows by score, and precompute the halved
squared norms xbar_i = x_i^T x_i / 2.

Query (Algorithm 2, Section 3.2): centre the query, score it, cut the
contiguous candidate window J = {j : |alpha_j - alpha_q| <= R} by binary
search (valid by the Cauchy-Schwarz bound eq. (lower)), evaluate
t_j = xbar_j - x_j^T x_q for j in J (eq. (ip2); Section 4 notes this is a
gemv, or a gemm over the union window for several queries), and keep the j
with t_j <= (R^2 - x_q^T x_q)/2.

Readings where the paper is silent or its floating-point claim does not
hold (each one is listed in the design notes):

* The paper treats the scores as exact.  Here the window is widened outward
  by a rigorous bound on the rounding of the computed scores, so that it is a
  superset of the exact-arithmetic window; extra candidates are harmless.
* Section 4 claims the decomposition has the same relative error bound as
  the direct form.  Under cancellation its error scales with
  (||x_j|| + ||x_q||)^2, not with the distance.  Decisions whose decomposed
  value lies within a rigorous absolute error bound of R^2 are therefore
  re-taken with the normative direct form on the original coordinates, so
  the result equals O1's exactly.  ``literal=True`` skips that band and
  reproduces the printed algorithm as a diagnostic.
* Sign of v1: the entry of largest magnitude is made positive (an SVD leaves
  it arbitrary; the result set does not depend on it).
"""

from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .brute import Neighbors, normative_sqdist

U64 = 2.0**-53  # unit roundoff of float64


def _gamma(k: int) -> float:
    """gamma_k = k u / (1 - k u), Section 4 (Higham, Lemma 3.1)."""
    return k * U64 / (1.0 - k * U64)


def first_principal_component(X: np.ndarray, svd_limit: int = 10_000_000) -> np.ndarray:
    """First right singular vector of the centred matrix X (eq. (svd)).

    For n*d up to ``svd_limit`` a thin SVD of X is used; beyond it the top
    eigenvector of X^T X, which has the same right singular vectors.  The
    largest-magnitude entry is made positive.  A zero matrix gives e_1.
    """
    n, d = X.shape
    if n == 0 or not np.any(X):
        v = np.zeros(d)
        v[0] = 1.0
        return v
    if n * d <= svd_limit:
        _, _, vt = np.linalg.svd(X, full_matrices=False)
        v = vt[0].copy()
    else:
        w, V = np.linalg.eigh(X.T @ X)
        v = V[:, np.argmax(w)].copy()
    if v[np.argmax(np.abs(v))] < 0:
        v = -v
    return v


@dataclass
class SnnIndex:
    mu: np.ndarray  # (d,) mean of the data
    v: np.ndarray  # (d,) sorting direction (v1 unless supplied)
    X: np.ndarray  # (n, d) centred rows in score order
    P: np.ndarray  # (n, d) original rows (float64) in score order
    alpha: np.ndarray  # (n,) sorted scores
    xbar: np.ndarray  # (n,) halved squared norms in score order
    xnorm: np.ndarray  # (n,) ||x_i|| in score order
    order: np.ndarray  # (n,) int64: sorted position -> original row id
    eps_max: float  # bound on |alpha_i - v.(p_i - mu)| over all i


def build_index(P, v=None) -> SnnIndex:
    """Algorithm 1.  ``v`` overrides the principal component (any nonzero
    vector keeps the query exact, by eq. (lower))."""
    P = np.ascontiguousarray(np.asarray(P), dtype=np.float64)
    n, d = P.shape
    mu = P.mean(axis=0)  # step 2
    X = P - mu  # step 3
    if v is None:
        v = first_principal_component(X)  # step 4
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(d))
    alpha = X @ v  # step 5
    order = np.argsort(alpha, kind="stable")  # step 6
    X = X[order]
    alpha = alpha[order]
    xbar = 0.5 * np.einsum("ij,ij->i", X, X)  # step 7
    xnorm = np.sqrt(2.0 * xbar)
    vnorm = float(np.linalg.norm(v))
    # |fl(x_i . v) - (p_i - mu).v| <= (u + gamma_d) ||x_i|| ||v||, padded.
    eps_max = 1.01 * _gamma(d + 2) * float(xnorm.max(initial=0.0)) * vnorm
    return SnnIndex(mu, v, X, P[order], alpha, xbar, xnorm, order, eps_max)


def _window(index: SnnIndex, aq: np.ndarray, qnorm: np.ndarray, R: float, d: int):
    """Step 4: [lo, hi) of sorted positions with |alpha_j - alpha_q| <= W_q.

    W_q widens R*||v|| outward so that every j with S(p_j, q) <= fl(R*R) is
    inside: S >= (1 - gamma_{d+2}) S* and fl(R*R) <= (1 + u) R^2 bound the
    exact distance, and eps_j, eps_q bound the score rounding.
    """
    vnorm = float(np.linalg.norm(index.v))
    eps_q = 1.01 * _gamma(d + 2) * qnorm * vnorm
    W = (R * vnorm * (1.0 + 4.0 * _gamma(d + 3)) + index.eps_max + eps_q) * (1.0 + 8 * U64)
    lo_v = np.nextafter(aq - W, -np.inf)
    hi_v = np.nextafter(aq + W, np.inf)
    lo = np.searchsorted(index.alpha, lo_v, side="left")
    hi = np.searchsorted(index.alpha, hi_v, side="right")
    return lo, hi


def query(index: SnnIndex, Q, R: float, block: int = 64, literal: bool = False, R2=None):
    """Algorithm 2 for every row of Q.  Returns (Neighbors, stats).

    block == 1 runs one gemv per query as printed; block > 1 sorts the
    queries by score and evaluates blocks of ``block`` score-adjacent
    queries with one gemm over their union window (Section 4), keeping for
    each query only its own window.  Both give the same result.

    stats: pairs_window = sum_q |J_q|, band = pairs re-decided with the
    normative S, literal_diff = pairs where the printed test (no band)
    would decide differently.

    R2: the squared threshold S is compared with (default fl(R*R)); when
    given, R must satisfy R^2 >= R2 exactly, since the window is cut with R.
    """
    Q = np.ascontiguousarray(np.asarray(Q), dtype=np.float64)
    m, d = Q.shape
    if d != index.X.shape[1]:
        raise ValueError("query dimension differs from the index")
    R = float(R)
    if not np.isfinite(R) or R < 0:
        raise ValueError("R must be finite and >= 0")
    if R2 is None:
        R2 = R * R
    elif not (0.0 <= float(R2) and Fraction(R) ** 2 >= Fraction(float(R2))):
        raise ValueError("R2 must be >= 0 and at most R^2")
    R2 = float(R2)
    xq = Q - index.mu  # step 2
    aq = xq @ index.v  # step 3
    qn2 = np.einsum("ij,ij->i", xq, xq)
    qnorm = np.sqrt(qn2)
    lo, hi = _window(index, aq, qnorm, R, d)  # step 4
    g = _gamma(d + 3)
    rows_ids = [None] * m
    rows_S = [None] * m
    band_total = 0
    literal_diff = 0
    qorder = np.argsort(aq, kind="stable") if block > 1 else np.arange(m)
    for b0 in range(0, m, max(block, 1)):
        qs = qorder[b0 : b0 + max(block, 1)]
        J0, J1 = int(lo[qs].min()), int(hi[qs].max())
        if J1 <= J0:
            for q in qs:
                rows_ids[q] = np.zeros(0, np.int64)
                rows_S[q] = np.zeros(0)
            continue
        XJ = index.X[J0:J1]
        G = XJ @ xq[qs].T  # step 5 (gemv / gemm of Section 4)
        T = index.xbar[J0:J1, None] - G
        for c, q in enumerate(qs):
            a, b = int(lo[q]) - J0, int(hi[q]) - J0
            if b <= a:
                rows_ids[q] = np.zeros(0, np.int64)
                rows_S[q] = np.zeros(0)
                continue
            t = T[a:b, c]
            s_dec = 2.0 * t + qn2[q]  # ||x_j - x_q||^2 by eq. (ip2)
            keep_lit = t <= (R2 - qn2[q]) / 2.0  # step 6 as printed
            if literal:
                keep = keep_lit
            else:
                nj = index.xnorm[J0 + a : J0 + b]
                E = 4.0 * g * ((nj + qnorm[q]) ** 2 + R2)
                band = np.abs(s_dec - R2) <= E
                keep = s_dec <= R2
                bi = np.flatnonzero(band)
                band_total += bi.size
                if bi.size:
                    S_b = normative_sqdist(index.P[J0 + a + bi], Q[q])
                    keep[bi] = S_b <= R2
                literal_diff += int(np.count_nonzero(keep != keep_lit))
            sel = np.flatnonzero(keep) + J0 + a
            rows_ids[q] = index.order[sel]
            rows_S[q] = normative_sqdist(index.P[sel], Q[q]) if sel.size else np.zeros(0)
    counts = np.array([r.size for r in rows_ids], dtype=np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols, dists = [], []
    for q in range(m):
        o = np.argsort(rows_ids[q], kind="stable")
        cols.append(rows_ids[q][o].astype(np.int32))
        dists.append(np.sqrt(rows_S[q][o]).astype(np.float32))
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    dist = np.concatenate(dists) if dists else np.zeros(0, np.float32)
    stats = {
        "pairs_window": int(np.sum(hi - lo)),
        "band": int(band_total),
        "literal_diff": int(literal_diff),
        "lo": lo,
        "hi": hi,
    }
    return Neighbors(row_ptr, col.astype(np.int32), dist.astype(np.float32)), stats
