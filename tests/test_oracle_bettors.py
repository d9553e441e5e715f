"""Pins of the cheap in-play bettor rules (oracle/bettors.py, paper
Section 5) and of the race trace they read (oracle race_trace, Section 3):
hand-worked views, the exact-ratio reading of LinEx checked with integer
arithmetic, ZI's uniform choice checked bit by bit for powers of two, and
the trace checked against the step count of the same simulation and
against the in-play state generator."""
import numpy as np
import pytest

from oracle import bettors as B

L100 = 100.0


def test_leader_and_second_ties_go_to_lowest_index():
    x = np.float32([3, 5, 5, 1])
    assert B.leader(x) == 1
    assert B.second(x, 1) == 2
    assert B.view(B.LW, 0.0, [x], 0, L100, 0, 0, 1) == 1


def test_underdog_threshold_by_hand():
    tr = [np.float32([10, 12, 9.5])]
    # leader 1 at 12, second 0 at 10: distance 2
    assert B.view(B.UD, 3.0, tr, 0, L100, 0, 0, 1) == 0
    assert B.view(B.UD, 2.0, tr, 0, L100, 0, 0, 1) == 1   # not strictly below D
    assert B.view(B.UD, 2.0000002, tr, 0, L100, 0, 0, 1) == 0
    assert B.view(B.UD, 0.0, tr, 0, L100, 0, 0, 1) == 1
    assert B.view(B.UD, 5.0, [np.float32([7.0])], 0, L100, 0, 0, 1) == 0
    # equal leaders: P1 is index 0, P2 index 2, distance 0 < D picks P2
    assert B.view(B.UD, 1.0, [np.float32([4, 1, 4])], 0, L100, 0, 0, 1) == 2


def test_linex_by_hand():
    # comp 0 leads and moves 5 a tick; comp 1 is 5 behind but moves 6 a tick,
    # after a slow first tick (4 du)
    tr = np.float32([[35, 35], [40, 39], [45, 45], [50, 51]])
    L = 100.0
    # row 3, N=1: disp (5, 6), rem (50, 49): comp 1 wins (8.2 vs 10 ticks)
    assert B.view(B.LINEX, 1, tr, 3, L, 0, 0, 1) == 1
    # N=3: disp (15, 16): ratios 50/15 = 3.33, 49/16 = 3.06: still comp 1
    assert B.view(B.LINEX, 3, tr, 3, L, 0, 0, 1) == 1
    # row 1, N=1: disp (5, 4), rem (60, 61): comp 0
    assert B.view(B.LINEX, 1, tr, 1, L, 0, 0, 1) == 0
    # window longer than the trace: w = min(N, r)
    assert B.view(B.LINEX, 50, tr, 1, L, 0, 0, 1) == 0
    assert B.view(B.LINEX, 50, tr, 3, L, 0, 0, 1) == B.view(B.LINEX, 3, tr, 3, L, 0, 0, 1)
    # row 0 has no history: LW's view (tie at 35 -> comp 0)
    assert B.view(B.LINEX, 4, tr, 0, L, 0, 0, 1) == 0


def test_linex_window_is_the_whole_trace_when_n_exceeds_it():
    # over both ticks comp 0 is faster (12 vs 9 du), over the last tick comp 1 (8 vs 2)
    tr = np.float32([[0, 5], [10, 6], [12, 14]])
    L = 100.0
    assert B.view(B.LINEX, 50, tr, 2, L, 0, 0, 1) == 0  # w = min(50, 2) = 2
    assert B.view(B.LINEX, 2, tr, 2, L, 0, 0, 1) == 0
    assert B.view(B.LINEX, 1, tr, 2, L, 0, 0, 1) == 1


def test_linex_window_changes_the_pick():
    # comp 1 had a fast first tick, then slowed down
    tr = np.float32([[35, 30], [40, 39], [45, 44]])
    L = 100.0
    # N=1: disp (5, 5), rem (55, 56): comp 0
    assert B.view(B.LINEX, 1, tr, 2, L, 0, 0, 1) == 0
    # N=2: disp (10, 14), rem (55, 56): 5.5 vs 4 ticks: comp 1
    assert B.view(B.LINEX, 2, tr, 2, L, 0, 0, 1) == 1


def test_linex_equal_ratios_and_no_motion():
    L = 10.0
    tr = np.float32([[2, 6], [4, 7]])
    # rem (6, 3), disp (2, 1): both 3 ticks: lowest index, not the leader
    assert B.view(B.LINEX, 1, tr, 1, L, 0, 0, 1) == 0
    # a competitor that did not move is never picked by LinEx
    tr = np.float32([[2, 7], [4, 7]])
    assert B.view(B.LINEX, 1, tr, 1, L, 0, 0, 1) == 0
    # nobody moved: LW's view
    tr = np.float32([[2, 7], [2, 7]])
    assert B.view(B.LINEX, 1, tr, 1, L, 0, 0, 1) == 1


def _exact_less(rem_a, disp_a, rem_b, disp_b):
    """rem_a/disp_a < rem_b/disp_b by integer cross-multiplication of the
    binary fractions of the single-precision values."""
    na, da = float(rem_a).as_integer_ratio()
    ma, ea = float(disp_a).as_integer_ratio()
    nb, db = float(rem_b).as_integer_ratio()
    mb, eb = float(disp_b).as_integer_ratio()
    # (na/da)/(ma/ea) < (nb/db)/(mb/eb)  <=>  na*ea*db*mb < nb*eb*da*ma  (all > 0)
    return na * ea * db * mb < nb * eb * da * ma


def test_linex_compares_exact_ratios_not_rounded_quotients():
    """Two-competitor windows whose single-precision quotients rem/disp are
    equal although the exact ratios differ: the pick must follow the exact
    order.  Positions lie in [512, 1024) below a line at 1024, so both
    differences are exact (Sterbenz) and the ratios are those of the trace."""
    L = np.float32(1024.0)
    u = np.float32(2.0 ** -14)  # spacing of single precision in [512, 1024)
    xa, ba = np.float32(700.0), np.float32(690.0)
    qa = np.float32(np.float32(L - xa) / np.float32(xa - ba))
    i = np.arange(-600, 600, dtype=np.float32)
    xb = (np.float32(xa) + i[:, None] * u).astype(np.float32) + np.zeros((1, i.size), np.float32)
    bb = (np.float32(ba) + i[None, :] * u).astype(np.float32) + np.zeros((i.size, 1), np.float32)
    qb = np.float32(L - xb) / np.float32(xb - bb)
    cand = np.argwhere(qb == qa)
    hits = 0
    for r, c in cand:
        x1, b1 = xb[r, c], bb[r, c]
        rem = (np.float32(L - xa), np.float32(L - x1))
        disp = (np.float32(xa - ba), np.float32(x1 - b1))
        if _exact_less(rem[1], disp[1], rem[0], disp[0]):
            tr = np.float32([[ba, b1], [xa, x1]])
            assert B.view(B.LINEX, 1, tr, 1, float(L), 0, 0, 1) == 1
            hits += 1
        elif _exact_less(rem[0], disp[0], rem[1], disp[1]):
            tr = np.float32([[b1, ba], [x1, xa]])  # competitor 1 holds the smaller ratio
            assert B.view(B.LINEX, 1, tr, 1, float(L), 0, 0, 1) == 1
            hits += 1
        if hits >= 20:
            break
    assert hits >= 5


def test_zi_power_of_two_is_the_top_bits():
    from oracle import philox4x32_10
    seed = 0x0123456789ABCDEF
    for n, k in ((1, 0), (2, 1), (4, 2), (16, 4)):
        for t in range(3):
            for b in range(50):
                w = int(philox4x32_10([t, b, 0xFFFFFFFF, 0xFFFFFFFF],
                                      [seed & 0xFFFFFFFF, seed >> 32])[0])
                want = w >> (32 - k) if k else 0
                assert B.zi_pick(seed, t, b, n) == want


def test_zi_is_uniform_and_fresh_each_tick():
    n, T, nb = 7, 40, 500
    picks = np.array([[B.zi_pick(99, t, b, n) for b in range(nb)] for t in range(T)])
    assert picks.min() == 0 and picks.max() == n - 1
    counts = np.bincount(picks.ravel(), minlength=n)
    e = picks.size / n
    chi2 = float(((counts - e) ** 2 / e).sum())
    assert chi2 < 22.5  # 6 degrees of freedom, p ~ 0.001
    # a bettor's view changes between ticks (fresh draw) for most bettors
    assert (picks[0] != picks[1]).mean() > 0.7


def test_views_counts_match_views():
    rng = np.random.default_rng(3)
    tr = np.cumsum(np.float32(rng.uniform(1, 3, (12, 5))), axis=0, dtype=np.float32)
    kinds = np.array([0, 1, 2, 3] * 6, np.uint8)
    params = np.float32([0, 0, 1.5, 3] * 6)
    v, c = B.views(kinds, params, tr, 100.0, 7, 11, first_row=2, n_eval=9)
    assert v.shape == (9, 24) and c.shape == (9, 5)
    for i in range(9):
        np.testing.assert_array_equal(np.bincount(v[i], minlength=5), c[i])
    # LW bettors all hold the leader's index
    for i in range(9):
        assert (v[i, kinds == B.LW] == B.leader(tr[2 + i])).all()


# ------------------------------------------------------------------ trace

def _race(n, seed=4):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(2.0, 4.0, n)
    hi = lo + rng.uniform(1.0, 6.0, n)
    comp = np.stack([lo, hi, rng.uniform(0.8, 1.0, n), rng.uniform(-0.2, 0.2, n),
                     rng.uniform(0.0, 2.0, n)], axis=1).astype(np.float32)
    return comp


@pytest.mark.parametrize("n,sim", [(1, 0), (3, 5), (8, 2), (20, 9)])
def test_trace_rows_equal_ticks_to_first_finish(orc, n, sim):
    comp, L = _race(n), 300.0
    tr = orc.race_trace(comp, L, seed=21, request=3, sim=sim, max_rows=100000)
    assert (tr[0] == 0).all()
    assert (tr < L).all() and (np.diff(tr, axis=0) > 0).all()
    # the same simulation run to its first finisher: every competitor steps
    # every tick up to and including the crossing tick
    _, _, steps = orc.race_sim(comp, L, 1, seed=21, request=3, sim_begin=sim, stop_after=1)
    assert steps % n == 0 and steps // n == tr.shape[0]


def test_trace_rows_equal_prefix_states(orc):
    comp, L = _race(6, seed=8), 250.0
    state = orc.race_prefix(comp, L, 5, 1, 2, 40.0)
    tr = orc.race_trace(comp, L, 5, 1, 2, 100000, state=state)
    np.testing.assert_array_equal(tr[0], state[1])
    for r in (1, 2, 7, tr.shape[0] // 2, tr.shape[0] - 1):
        t, pos, _ = orc.race_prefix(comp, L, 5, 1, 2, float(tr[r].max()), state=state)
        assert t == state[0] + r
        np.testing.assert_array_equal(pos, tr[r])
    short = orc.race_trace(comp, L, 5, 1, 2, 4, state=state)
    np.testing.assert_array_equal(short, tr[:4])


def test_rp_views_by_hand():
    wins = np.array([[0, 3, 1, 3], [5, 0, 0, 0], [0, 0, 0, 0], [1, 2, 3, 4], [9, 9, 9, 99]],
                    np.uint64)
    v, c = B.rp_views(wins, 3)  # competitor 3 is outside the race's first 3 columns
    assert v.tolist() == [1, 0, 0, 2, 0]
    assert c.tolist() == [3, 1, 1]
    v4, _ = B.rp_views(wins, 4)
    assert v4.tolist() == [1, 0, 0, 3, 3]
