"""The C oracle against an independent exact enumeration of tiny races
(oracle/enumerate.py): identical finish order and identical consumed draws
for every draw sequence, and Monte-Carlo frequencies within 5 sigma of the
exact probability mass function over finish orders (paper Section 6)."""
import numpy as np
import pytest

from oracle.enumerate import draws_matrix, enumerate_race

L_TINY = 4.0

# (name, comp rows (lo, hi, pref, rho, theta[, gamma, tau]), K, L, stop_after)
CASES = [
    ("n2_k4_free", [[1, 2, 1, 0, 0], [1, 2, 1, 0, 0]], 4, 3.0, None),
    ("n2_k4_block", [[1, 2, 1, 0, 0.5], [1, 2, 1, 0, 1.0]], 4, 3.0, None),
    ("n3_k2_mixed_rho", [[1, 2, 1, 0, 0.5], [1, 2, 1, 0.2, 0.5], [1, 2, 1, -0.2, 0]], 2, 4.0, None),
    ("n3_k2_pref", [[1, 2, 0.75, 0, 1.0], [1, 3, 1, 0.1, 0.5], [1.5, 2, 1, 0, 0]], 2, 4.0, None),
    ("n4_k2_block", [[1, 2, 1, 0, 0.5], [1, 2, 1, 0, 0.5], [1, 2, 1, 0.2, 1.0], [1, 2, 1, -0.2, 0.5]], 2, 3.0, None),
    ("n4_k2_winner_only", [[1, 2, 1, 0, 0.5], [1, 2, 1, 0, 0.5], [1, 2, 1, 0.2, 1.0], [1, 2, 1, -0.2, 0.5]], 2, 4.0, 1),
    ("n3_k2_time_term", [[1, 2, 1, 0, 0.5, 0.125, 2], [1, 2, 1, 0.2, 0.5, -0.0625, 3],
                         [1, 2, 1, -0.2, 0, 0, 0]], 2, 4.0, None),
]


@pytest.mark.parametrize("name,comp,K,L,stop", CASES, ids=[c[0] for c in CASES])
def test_every_path_matches(orc, name, comp, K, L, stop):
    comp = np.array(comp, np.float32)
    n = comp.shape[0]
    pmf, paths = enumerate_race(comp, L, K, stop_after=stop)
    assert sum(pmf.values()) == 1
    ticks = 1 + max([t for p in paths for (t, _) in p[0]] + [0]) + 1
    D = draws_matrix(paths, n, K, ticks)
    orders, used, trace = orc.race_draws(comp, L, D, stop_after=stop, return_used=True,
                                         return_trace=True)
    for i, (consumed, order, _, tr) in enumerate(paths):
        got = [int(x) for x in orders[i] if x != 0xFF]
        assert tuple(got) == order, (i, consumed)
        assert set(zip(*np.nonzero(used[i]))) == set(consumed.keys())
        # positions after every tick, bit for bit (finished competitors keep
        # their crossing position in both implementations)
        np.testing.assert_array_equal(trace[i, :len(tr)], np.array(tr, np.float32))


@pytest.mark.parametrize("name,comp,K,L,stop", CASES, ids=[c[0] for c in CASES])
def test_monte_carlo_matches_exact_pmf(orc, name, comp, K, L, stop):
    comp = np.array(comp, np.float32)
    pmf, _ = enumerate_race(comp, L, K, stop_after=stop)
    N = 400_000
    orders, wins, _ = orc.race_sim(comp, L, N, seed=2021, levels=K, stop_after=stop, threads=8)
    keys, counts = np.unique(orders, axis=0, return_counts=True)
    freq = {tuple(int(x) for x in k if x != 0xFF): c / N for k, c in zip(keys, counts)}
    assert set(freq) <= set(pmf)
    for order, p in pmf.items():
        p = float(p)
        sig = np.sqrt(p * (1 - p) / N)
        assert abs(freq.get(order, 0.0) - p) <= 5 * sig + 1e-12, (order, freq.get(order), p)
    assert wins.sum() == N


def test_time_term_paths_from_an_in_play_state(orc):
    """The time term reads the absolute tick: from a state at tick 5 the
    enumeration and the oracle agree path by path."""
    comp = np.array([[1, 2, 1, 0, 0.5, 0.0625, 7], [1, 2, 1, 0.1, 0.5, -0.03125, 9],
                     [1, 2, 1, 0, 0, 0.25, 6]], np.float32)
    state = (5, np.array([1.0, 1.5, 0.5], np.float32), np.array([1.0, 1.25, 1.5], np.float32))
    L, K = 5.0, 2
    pmf, paths = enumerate_race(comp, L, K, state=state)
    assert sum(pmf.values()) == 1
    ticks = 1 + max([t for p in paths for (t, _) in p[0]] + [0]) + 1
    D = draws_matrix(paths, 3, K, ticks)
    orders, used, trace = orc.race_draws(comp, L, D, state=state, return_used=True,
                                         return_trace=True)
    for i, (consumed, order, _, tr) in enumerate(paths):
        assert tuple(int(x) for x in orders[i] if x != 0xFF) == order
        assert set(zip(*np.nonzero(used[i]))) == set(consumed.keys())
        np.testing.assert_array_equal(trace[i, :len(tr)], np.array(tr, np.float32))
    # the same races without the time term take other paths
    pmf0, _ = enumerate_race(comp[:, :5], L, K, state=state)
    assert pmf0 != pmf
