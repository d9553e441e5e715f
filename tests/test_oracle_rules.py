"""Hand-worked cases of the step rule (tests/golden/race_rules.json) run on
the CPU oracle.  The same fixture drives the GPU rule tests."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "race_rules.json")
CASES = json.load(open(GOLDEN))["cases"]


def _state(case):
    st = case["state"]
    if st is None:
        return None
    return (st["tick"], np.array(st["pos"], np.float32), np.array(st["prev"], np.float32))


@pytest.mark.parametrize("case", [c for c in CASES if c["kind"] == "tick"], ids=lambda c: c["name"])
def test_single_tick(orc, case):
    comp = np.array(case["comp"], np.float32)
    st = _state(case)
    lead = np.float32(max(st[1]))
    target = np.nextafter(lead, np.float32(np.inf))
    t, pos, prev = orc.race_prefix(comp, case["L"], seed=99, request=0, sim=0, target=target, state=st)
    assert t == case["expect"]["tick"]
    np.testing.assert_array_equal(pos, np.array(case["expect"]["pos"], np.float32))
    np.testing.assert_array_equal(prev, np.array(case["expect"]["prev"], np.float32))


@pytest.mark.parametrize("case", [c for c in CASES if c["kind"] == "race"], ids=lambda c: c["name"])
def test_whole_race(orc, case):
    comp = np.array(case["comp"], np.float32)
    n = comp.shape[0]
    sims = 17
    orders, wins, steps = orc.race_sim(comp, case["L"], sims, seed=5, state=_state(case))
    exp = np.array(case["expect"]["order"], np.uint8)
    assert (orders == exp[None, :]).all()
    assert steps == sims * case["expect"]["steps_per_sim"]
    w = np.zeros(n, np.uint64)
    w[exp[0]] = sims
    np.testing.assert_array_equal(wins, w)
