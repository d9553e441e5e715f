"""GPU parity of the finish-order tallies: finish-position counts and the
PMF over complete orders, computed on the device from the kernel's own
finish-order matrix, equal the oracle's tallies of the oracle's orders."""
import math

import numpy as np
import pytest

from gpu_util import announce, require_gpu
from oracle import orders as O
from paper_2108_02419_amd import api, inputs
from paper_2108_02419_amd._bbe import Race

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("n,n_sims,stop", [(5, 1037, None), (7, 2000, None), (7, 500, 3),
                                           (3, 64, None), (20, 20_000, None), (12, 999, 5)])
def test_tallies_match_oracle(torch, orc, n, n_sims, stop):
    rng = np.random.default_rng(500 + n)
    comp = inputs.competitor_params(rng, n)
    announce(f"order tallies n={n} sims={n_sims} stop={stop}")
    race = Race(comp, inputs.TRACK_LEN)
    out = api.mc(race, n_sims, 8, request=n, stop_after=stop, want_orders=True)
    g_orders = out["orders"]
    rc = api.rank_counts(g_orders, n)
    pmf = api.order_pmf(g_orders, n) if n <= 7 else None
    torch.cuda.synchronize()
    o_orders, _, _ = orc.race_sim(comp, inputs.TRACK_LEN, n_sims, 8, request=n, stop_after=stop,
                                  threads=8)
    np.testing.assert_array_equal(g_orders.cpu().numpy(), o_orders)
    np.testing.assert_array_equal(rc.cpu().numpy().astype(np.uint64), O.rank_counts(o_orders, n))
    if pmf is not None:
        want = O.order_pmf(o_orders, n)
        np.testing.assert_array_equal(pmf.cpu().numpy().astype(np.uint64), want)
        assert pmf.shape[0] == math.factorial(n)
        if stop is None or stop == n:
            assert int(pmf.sum().item()) == n_sims


def test_empty_input(torch):
    e = torch.empty((0, 4), dtype=torch.uint8, device="cuda")
    rc = api.rank_counts(e, 4)
    pmf = api.order_pmf(e, 4)
    torch.cuda.synchronize()
    assert int(rc.abs().sum().item()) == 0 and int(pmf.abs().sum().item()) == 0
