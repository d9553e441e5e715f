"""Pins of the preference coefficient from race factors
(oracle/factors.py, paper Section 3): hand-worked products, the limits
the reading fixes (a perfect match and zero sensitivity leave the step
alone; full mismatch at sensitivity w leaves 1 - w), and independence of
the factors' contributions."""
import numpy as np
import pytest

from oracle.factors import pref_from_factors


def test_hand_worked():
    f = [0.5, 1.0, 0.0]
    p = [[0.25, 1.0, 0.5],    # 1 - 0.5*0.25 = 0.875; 1; 1 - 0.5*0.5 = 0.75 -> 0.65625
         [0.5, 0.0, 0.0]]     # 1; 1 - 0.75*1 = 0.25; 1 -> 0.25
    w = [[0.5, 0.75, 0.5],
         [0.5, 0.75, 0.5]]
    np.testing.assert_array_equal(pref_from_factors(f, p, w), np.float32([0.65625, 0.25]))


def test_limits():
    rng = np.random.default_rng(1)
    f = rng.uniform(0, 1, 6).astype(np.float32)
    p = rng.uniform(0, 1, (4, 6)).astype(np.float32)
    w = rng.uniform(0, 0.9, (4, 6)).astype(np.float32)
    assert (pref_from_factors(f, np.tile(f, (4, 1)), w) == 1).all()       # perfect match
    assert (pref_from_factors(f, p, np.zeros_like(w)) == 1).all()          # insensitive
    P = pref_from_factors([0.0], [[1.0]], [[0.375]])                       # full mismatch
    assert P[0] == np.float32(0.625)
    got = pref_from_factors(f, p, w)
    assert ((got > 0) & (got <= 1)).all()


def test_factors_multiply_independently():
    """With dyadic values every product is exact: P over two factors equals
    the product of P over each one alone, and the order does not matter."""
    f = np.float32([0.25, 0.75])
    p = np.float32([[0.75, 0.5]])
    w = np.float32([[0.5, 0.25]])
    both = pref_from_factors(f, p, w)[0]
    one = pref_from_factors(f[:1], p[:, :1], w[:, :1])[0]
    two = pref_from_factors(f[1:], p[:, 1:], w[:, 1:])[0]
    assert both == one * two == np.float32(0.75 * 0.9375)
    assert pref_from_factors(f[::-1], p[:, ::-1], w[:, ::-1])[0] == both


def test_underflow_rejected():
    F = 200
    with pytest.raises(ValueError):
        pref_from_factors(np.zeros(F), np.ones((1, F)), np.full((1, F), 0.999))
