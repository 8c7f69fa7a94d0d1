"""O3: exact rational fixed-radius search for tiny inputs.

Test infrastructure only (see the package docstring).

Every float is converted to the rational number it represents
(``fractions.Fraction(float)`` is exact), so S* = sum_k (p_k - q_k)^2 and
R*^2 are computed without rounding.  This is the mathematical definition of
the problem in Section 3 (all p_i with ||p_i - q|| <= R), against which the
normative float64 rule of O1 differs only for pairs whose exact squared
distance lies within the direct-form error bound gamma_{d+2} of Section 4
of R^2.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_sqdist(p, q) -> Fraction:
    """Exact ||p - q||^2 of two float vectors."""
    s = Fraction(0)
    for a, b in zip(np.asarray(p, dtype=np.float64).tolist(), np.asarray(q, dtype=np.float64).tolist()):
        t = Fraction(a) - Fraction(b)
        s += t * t
    return s


def exact_radius(P, Q, R: float):
    """Exact neighbour sets {i : ||p_i - q|| <= R} and the exact S* matrix.

    Returns (sets, S) where sets[r] is a sorted list of ids and S[r][i] is the
    Fraction S*(p_i, q_r).  Cost m*n*d rational operations: tiny inputs only.
    """
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    R2 = Fraction(float(R)) ** 2
    sets, S = [], []
    for q in Q:
        row = [exact_sqdist(p, q) for p in P]
        S.append(row)
        sets.append([i for i, s in enumerate(row) if s <= R2])
    return sets, S
