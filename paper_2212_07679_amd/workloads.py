"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the search
arithmetic, so both the HIP path's tests/bench and the CPU oracle can use it
without sharing any method code.  Every generator draws in float64 from
``numpy.random.default_rng([2212, 7679, tag])`` and casts to the workload's
dtype; the cast values are the data.

Workloads (sizes are the defaults; every generator takes smaller sizes for
parity tests):

uniform2d  n points uniform in [0,1]^2 (float64), m queries sampled from the
           data without replacement, R = 0.05 -- the synthetic setting of
           Section 6.1 (Table 1, d = 2).
gmm16      1e6 points, d = 16, float32: 20 isotropic clusters (std 1) with
           centres uniform in [-10,10]^16 and equal weights; 1e5
           out-of-sample queries from the same mixture; R = 1.5.
gmm128z    2e6 points, d = 128, float32: 50 clusters (std 0.5) with centres
           N(0, I), each feature then z-scored (the pre-processing of
           Section 6.4); self-query with R = 4.0.
batch256   256 independent instances, n log-uniform in [1e3, 1e5],
           d in {3, 8, 32}, uniform in the unit cube (float32), 10% of the
           points as queries, R giving ~30 expected neighbours under uniform
           density: R = (30 / ((n - 1) V_d))^(1/d), V_d the unit-ball volume.
blobs3d    5e6 points, d = 3, float32: 80% from 1,000 Gaussian blobs
           (std 0.01) with centres uniform in [0,1]^3, 20% uniform
           background; self-query with R = 0.005.
angular100 1,183,514 points, d = 100, float32 (the shape of the GloVe-100
           angular set of Section 6): directions clustered around 100 random
           unit centres (offset N(0, 0.7^2 I / d)), each row scaled by a
           log-normal length (raw embeddings are not unit vectors); 1e4
           out-of-sample queries from the same mixture; neighbours within an
           angle of 39 degrees (alpha; R is unset: the Euclidean radius on
           normalised rows follows from alpha).
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

SEED = (2212, 7679)


def rng_for(tag: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED[0], SEED[1], int(tag), int(sub)])


@dataclass
class Workload:
    name: str
    P: np.ndarray  # (n, d) data, C-contiguous, float32 or float64
    Q: Optional[np.ndarray]  # (m, d) queries; None = self-query (Q is P)
    R: float
    alpha: Optional[float] = None  # angular workloads: the angle (radians)

    @property
    def n(self) -> int:
        return self.P.shape[0]

    @property
    def d(self) -> int:
        return self.P.shape[1]

    @property
    def m(self) -> int:
        return self.n if self.Q is None else self.Q.shape[0]

    @property
    def queries(self) -> np.ndarray:
        return self.P if self.Q is None else self.Q


def uniform2d(n: int = 10_000, m: int = 1_000, R: float = 0.05, seed: int = 1) -> Workload:
    g = rng_for(1, seed)
    P = g.random((n, 2))
    Q = P[g.choice(n, size=min(m, n), replace=False)]
    return Workload("uniform2d", np.ascontiguousarray(P), np.ascontiguousarray(Q), R)


def _mixture(g: np.random.Generator, centres: np.ndarray, count: int, std: float) -> np.ndarray:
    lab = g.integers(0, centres.shape[0], size=count)
    return centres[lab] + std * g.standard_normal((count, centres.shape[1]))


def gmm16(n: int = 1_000_000, m: int = 100_000, R: float = 1.5, d: int = 16, k: int = 20, seed: int = 2) -> Workload:
    g = rng_for(2, seed)
    centres = g.uniform(-10.0, 10.0, size=(k, d))
    P = _mixture(g, centres, n, 1.0).astype(np.float32)
    Q = _mixture(g, centres, m, 1.0).astype(np.float32)
    return Workload("gmm16", P, Q, R)


def gmm128z(n: int = 2_000_000, R: float = 4.0, d: int = 128, k: int = 50, seed: int = 3) -> Workload:
    g = rng_for(3, seed)
    centres = g.standard_normal((k, d))
    P = _mixture(g, centres, n, 0.5)
    P -= P.mean(axis=0)
    P /= P.std(axis=0)  # ddof = 0
    return Workload("gmm128z", P.astype(np.float32), None, R)


def ball_volume(d: int) -> float:
    return math.pi ** (d / 2) / math.gamma(d / 2 + 1)


def batch_radius(n: int, d: int, expected: float = 30.0) -> float:
    return (expected / ((n - 1) * ball_volume(d))) ** (1.0 / d)


def batch256(count: int = 256, n_lo: float = 1e3, n_hi: float = 1e5, dims=(3, 8, 32), frac: float = 0.1, seed: int = 4) -> List[Workload]:
    g = rng_for(4, seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(dims[g.integers(0, len(dims))])
        P = g.random((n, d)).astype(np.float32)
        m = int(math.ceil(frac * n))
        Q = P[g.choice(n, size=m, replace=False)]
        out.append(Workload(f"batch256[{i}]", P, np.ascontiguousarray(Q), batch_radius(n, d)))
    return out


def blobs3d(n: int = 5_000_000, R: float = 0.005, k: int = 1000, blob_frac: float = 0.8, seed: int = 5) -> Workload:
    g = rng_for(5, seed)
    centres = g.random((k, 3))
    nb = int(round(blob_frac * n))
    B = _mixture(g, centres, nb, 0.01)
    U = g.random((n - nb, 3))
    P = np.concatenate([B, U])[g.permutation(n)]
    return Workload("blobs3d", P.astype(np.float32), None, R)


def gaussian_blob(n: int, d: int, s: float, seed: int = 6) -> np.ndarray:
    """Elongated Gaussian of Section 5: std [1, s, ..., s] per coordinate."""
    g = rng_for(6, seed)
    X = g.standard_normal((n, d))
    X[:, 1:] *= s
    return X


def lattice(lo: int, hi: int, d: int = 2) -> np.ndarray:
    """All integer points of [lo, hi]^d (float64), row-major order."""
    axes = [np.arange(lo, hi + 1, dtype=np.float64)] * d
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([gr.reshape(-1) for gr in grids], axis=1)


def angular100(n: int = 1_183_514, m: int = 10_000, d: int = 100, k: int = 100, spread: float = 0.7,
               alpha_deg: float = 39.0, seed: int = 7) -> Workload:
    g = rng_for(7, seed)
    C = g.standard_normal((k, d))
    C /= np.linalg.norm(C, axis=1, keepdims=True)

    def draw(count):
        lab = g.integers(0, k, size=count)
        X = C[lab] + spread * g.standard_normal((count, d)) / math.sqrt(d)
        return X * np.exp(0.3 * g.standard_normal((count, 1)))

    P = draw(n)
    Q = draw(m)
    return Workload("angular100", P.astype(np.float32), Q.astype(np.float32), float("nan"), math.radians(alpha_deg))
