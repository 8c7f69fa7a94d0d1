"""Planted mistakes in the oracle (CPU only) must be caught by its pins.

Each case swaps one internal routine of the oracle for a plausible wrong
version (a dropped term, a wrong sign, a strict comparison, a transposed
operand, a fused or reordered sum) and checks that at least one pin fails.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import brute as B
from paper_2212_07679_amd import workloads as W
from tests.test_oracle_exact import lattice_count


def pins_hold():
    """A compact set of the exact pins; raises AssertionError on failure."""
    P = W.lattice(-6, 6, 2)
    nb = oracle.brute_radius(P, np.zeros((1, 2)), 5.0)
    assert nb.row_ptr[-1] == 81
    # balls clipped by the lattice range: every coordinate of the centre
    # changes the count
    P = W.lattice(-3, 10, 2)
    nb = oracle.brute_radius(P, np.array([[8.0, 0.0]]), 5.0)
    assert nb.row_ptr[-1] == lattice_count(25, (8, 0), -3, 10, 2)
    P = W.lattice(-4, 8, 3)
    nb = oracle.brute_radius(P, np.array([[7.0, -3.0, 0.0]]), 3.0)
    assert nb.row_ptr[-1] == lattice_count(9, (7, -3, 0), -4, 8, 3)
    s = oracle.normative_sqdist(np.array([[2.0**-27, 2.0**-27, 1.0 + 2.0**-30]]), np.zeros(3))[0]
    assert s == 1.0 + 2.0**-29
    s = oracle.normative_sqdist(np.array([[1.0, 2.0**-27, 2.0**-27, 2.0**-27]]), np.zeros(4))[0]
    assert s == 1.0


def _drop_last(P, Qb):
    s = np.zeros((Qb.shape[0], P.shape[0]))
    for k in range(P.shape[1] - 1):
        t = P[None, :, k] - Qb[:, k, None]
        s += t * t
    return s


def _plus_sign(P, Qb):
    s = np.zeros((Qb.shape[0], P.shape[0]))
    for k in range(P.shape[1]):
        t = P[None, :, k] + Qb[:, k, None]
        s += t * t
    return s


def _wrong_index(P, Qb):
    s = np.zeros((Qb.shape[0], P.shape[0]))
    for k in range(P.shape[1]):
        t = P[None, :, k] - Qb[:, 0, None]
        s += t * t
    return s


def _abs_not_square(P, Qb):
    s = np.zeros((Qb.shape[0], P.shape[0]))
    for k in range(P.shape[1]):
        s += np.abs(P[None, :, k] - Qb[:, k, None])
    return s ** 2


def _strict(P, Qb):
    s = B._orig_block(P, Qb)
    return np.nextafter(s, np.inf)  # behaves like a strict comparison at ties


def _reversed_sum(p, q):
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64).reshape(-1)
    s = np.zeros(p.shape[0])
    for k in reversed(range(p.shape[1])):
        t = p[:, k] - q[k]
        s += t * t
    return s


def _fused_sum(p, q):
    # emulate a fused multiply-add with exact rationals
    from fractions import Fraction
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64).reshape(-1)
    out = np.zeros(p.shape[0])
    for i in range(p.shape[0]):
        s = 0.0
        for k in range(p.shape[1]):
            t = float(p[i, k] - q[k])
            s = float(Fraction(s) + Fraction(t) * Fraction(t))
        out[i] = s
    return out


B._orig_block = B._block_sqdist


@pytest.mark.parametrize("mutant", [_drop_last, _plus_sign, _wrong_index, _abs_not_square, _strict])
def test_block_mutants_caught(monkeypatch, mutant):
    pins_hold()  # the real oracle passes
    monkeypatch.setattr(B, "_block_sqdist", mutant)
    with pytest.raises(AssertionError):
        pins_hold()


@pytest.mark.parametrize("mutant", [_reversed_sum, _fused_sum])
def test_sum_mutants_caught(monkeypatch, mutant):
    monkeypatch.setattr(oracle, "normative_sqdist", mutant)
    with pytest.raises(AssertionError):
        pins_hold()


def test_o2_without_band_caught():
    # the printed decomposition test without the band fails the cancellation pin
    g = np.random.default_rng(9)
    P = np.concatenate([1e8 + g.standard_normal((300, 3)) * 0.05,
                        -1e8 + g.standard_normal((300, 3)) * 0.05])
    Q = P[::7] + 0.01 * g.standard_normal((P[::7].shape[0], 3))
    ref = oracle.brute_radius(P, Q, 0.1)
    lit, _ = oracle.snn_query(oracle.build_index(P), Q, 0.1, literal=True)
    assert not (np.array_equal(ref.row_ptr, lit.row_ptr) and np.array_equal(ref.col, lit.col))


def test_o2_unwidened_window_caught(monkeypatch):
    # A window cut at exactly R*||v|| on rounded scores can miss a neighbour at
    # distance exactly R along the sorting direction; collinear lattice data
    # puts neighbours exactly there.
    from oracle import snn as S

    def narrow(index, aq, qnorm, R, d):
        lo = np.searchsorted(index.alpha, aq - R, side="left")
        hi = np.searchsorted(index.alpha, aq + R, side="left")  # drops alpha == aq + R
        return lo, hi

    t = np.arange(-50, 51, dtype=np.float64)
    P = np.stack([t, np.zeros_like(t)], 1)
    Q = P[::5]
    ref = oracle.brute_radius(P, Q, 3.0)
    good, _ = oracle.snn_query(oracle.build_index(P), Q, 3.0)
    assert np.array_equal(ref.col, good.col)
    monkeypatch.setattr(S, "_window", narrow)
    bad, _ = oracle.snn_query(oracle.build_index(P), Q, 3.0)
    assert not np.array_equal(ref.col, bad.col)
