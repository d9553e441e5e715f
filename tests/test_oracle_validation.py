"""Argument validation of the CPU oracle (the same rules bind the GPU
library's C ABI)."""
import numpy as np
import pytest

GOOD = np.array([[5.0, 8.0, 1.0, 0.1, 2.0]] * 3, np.float32)


def _bad_comp(col, val):
    c = GOOD.copy()
    c[1, col] = val
    return c


@pytest.mark.parametrize("comp", [
    _bad_comp(0, 0.0), _bad_comp(0, -1.0), _bad_comp(1, 4.0), _bad_comp(2, 0.0), _bad_comp(2, 1.5),
    _bad_comp(3, 1.0), _bad_comp(3, -1.0), _bad_comp(4, -0.5), _bad_comp(0, np.nan),
    _bad_comp(1, np.inf), np.zeros((0, 5), np.float32), np.repeat(GOOD[:1], 21, axis=0),
    _bad_comp(0, 1e-4),  # too slow: the race could not end within the tick bound
])
def test_bad_competitors_rejected(orc, comp):
    with pytest.raises(orc.OracleError):
        orc.race_sim(comp, 2000.0, 10, 1)


GOOD7 = np.array([[5.0, 8.0, 1.0, 0.1, 2.0, 0.001, 300.0]] * 3, np.float32)


def _bad_pace(col, val):
    c = GOOD7.copy()
    c[1, col] = val
    return c


@pytest.mark.parametrize("comp", [
    _bad_pace(5, np.nan), _bad_pace(5, np.inf), _bad_pace(6, -1.0), _bad_pace(6, 2.5),
    _bad_pace(6, 2.0**25), _bad_pace(6, np.nan),
    _bad_pace(5, -0.003),  # 1 - 0.1 - 0.9 = 0: the time term would stop the competitor
])
def test_bad_time_terms_rejected(orc, comp):
    with pytest.raises(orc.OracleError):
        orc.race_sim(comp, 2000.0, 10, 1)


def test_time_term_accepted_and_zero_is_the_plain_race(orc):
    ok = _bad_pace(5, -0.0029)  # R stays >= 1 - 0.1 - 0.87 = 0.03
    orc.race_sim(ok, 2000.0, 10, 1)
    plain = orc.race_sim(GOOD, 2000.0, 300, 4)
    zero = GOOD7.copy()
    zero[:, 5] = 0.0
    same = orc.race_sim(zero, 2000.0, 300, 4)
    for a, b in zip(plain, same):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("kw", [
    dict(L=0.0), dict(L=-5.0), dict(L=np.inf), dict(n_sims=0), dict(stop_after=0),
    dict(stop_after=4), dict(sim_begin=2**32 - 5, n_sims=10),
    dict(state=(3, np.array([0, 10, 2000], np.float32), np.ones(3, np.float32))),
    dict(state=(3, np.array([0, -1, 20], np.float32), np.ones(3, np.float32))),
    dict(state=(3, np.array([0, 1, 20], np.float32), np.array([1, 0, 1], np.float32))),
    dict(state=(3, np.array([0, 1, np.nan], np.float32), np.ones(3, np.float32))),
    dict(state=(2**32 - 10, np.zeros(3, np.float32), np.ones(3, np.float32))),
])
def test_bad_calls_rejected(orc, kw):
    args = dict(L=2000.0, n_sims=10, sim_begin=0, stop_after=None, state=None)
    args.update(kw)
    with pytest.raises(orc.OracleError):
        orc.race_sim(GOOD, args["L"], args["n_sims"], 1, sim_begin=args["sim_begin"],
                     stop_after=args["stop_after"], state=args["state"])


def test_good_call_accepted(orc):
    orc.race_sim(GOOD, 2000.0, 10, 1, sim_begin=2**32 - 10)
