"""Statistical pins of the oracle against closed forms and the paper's tables.

* Uniform data in the unit square / cube: the probability that two
  independent points lie within distance R <= 1 has the closed forms
      F_2(R) = pi R^2 - 8 R^3 / 3 + R^4 / 2,
      F_3(R) = 4 pi R^3 / 3 - 3 pi R^4 / 2 + 8 R^5 / 5 - R^6 / 6
  (integrate the product of triangular difference densities over the ball).
  The self-query return ratio excluding the query point itself estimates
  F_d(R); the ratios printed in Table 1 (d = 2) and Table 2 (d = 3) are such
  estimates on the paper's own samples (golden fixtures).
* The elongated Gaussian model of Section 5: the window probability
  P_1(c, R) and the hit probability P_2(c, R, s, d).
Tolerances are several standard deviations of the estimators.
"""

import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from paper_2212_07679_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def F2(R):
    return math.pi * R**2 - 8 * R**3 / 3 + R**4 / 2


def F3(R):
    return 4 * math.pi * R**3 / 3 - 3 * math.pi * R**4 / 2 + 8 * R**5 / 5 - R**6 / 6


def load(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            n, R, pct = line.split()
            rows.append((int(n), float(R), float(pct) / 100.0))
    return rows


def ratio_excluding_self(P, R):
    idx = oracle.build_index(P)
    nb, _ = oracle.snn_query(idx, P, R)
    n = P.shape[0]
    return (nb.row_ptr[-1] - n) / (n * (n - 1.0))


def tol(F, n):
    # U-statistic standard deviation bound: Var <= 4 F^2 / n + 2 F / n^2
    return 5.0 * math.sqrt(4 * F * F / n + 2 * F / (n * n))


@pytest.mark.parametrize("n,R,pct", load("table1_d2_ratios.txt"))
def test_table1_uniform_square(n, R, pct):
    P = np.random.default_rng([2212, 7679, 100, n, int(R * 1000)]).random((n, 2))
    F = F2(R)
    r = ratio_excluding_self(P, R)
    assert abs(r - F) <= tol(F, n)
    # the printed ratio is another sample of the same estimator
    assert abs(pct - F) <= tol(F, n)


@pytest.mark.parametrize("n,R,pct", load("table2_d3_ratios.txt"))
def test_table2_uniform_cube(n, R, pct):
    P = np.random.default_rng([2212, 7679, 101, n, int(R * 1000)]).random((n, 3))
    F = F3(R)
    r = ratio_excluding_self(P, R)
    assert abs(r - F) <= tol(F, n)
    # printed to two significant digits
    assert abs(pct - F) <= tol(F, n) + 0.05 * F


def test_table1_excludes_self():
    # At n = 2000, R = 0.02 the printed 0.1243 % matches F_2 = 0.1235 % and not
    # F_2 + 1/n = 0.1735 %: the paper's ratio does not count the query point.
    n, R, pct = 2000, 0.02, 0.001243
    assert abs(pct - F2(R)) <= tol(F2(R), n)
    assert abs(pct - (F2(R) + 1.0 / n)) > tol(F2(R), n)


def _P1(c, R):
    return stats.norm.cdf(c + R) - stats.norm.cdf(c - R)


def _P2(c, R, s, d):
    f = lambda r: stats.norm.pdf(r) * stats.chi2.cdf(max(R * R - (r - c) ** 2, 0.0) / (s * s), d - 1)
    val, _ = integrate.quad(f, c - R, c + R)
    return val


@pytest.mark.parametrize("c,R", [(0.0, 0.5), (0.8, 0.5), (1.5, 1.0)])
def test_elongated_gaussian_model(c, R):
    n, d, s = 100_000, 4, 0.4
    X = W.gaussian_blob(n, d, s, seed=21)
    q = np.zeros((1, d))
    q[0, 0] = c
    idx = oracle.build_index(X)
    nb, st = oracle.snn_query(idx, q, R, block=1)
    p1, p2 = _P1(c, R), _P2(c, R, s, d)
    win = (st["hi"][0] - st["lo"][0]) / n
    hits = nb.row_ptr[-1] / n
    # window: binomial noise plus the sample principal direction and mean
    assert abs(win - p1) <= 5 * math.sqrt(p1 * (1 - p1) / n) + 0.01
    assert abs(hits - p2) <= 5 * math.sqrt(p2 * (1 - p2) / n) + 1e-4
    assert p2 <= p1 + 1e-12
