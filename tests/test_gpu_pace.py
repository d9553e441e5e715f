"""GPU parity of races whose responsiveness carries a time term
(R = alpha + beta*d + gamma*min(t, tau), paper Section 3's R_c(t, d)):
finish orders, win counts and step counts of the paced kernels bit-exact
against the oracle, from the start and in play, alone and mixed with plain
races in one batch; traces and in-play states as well."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from paper_2108_02419_amd import api, inputs
from paper_2108_02419_amd._bbe import BatchPlan, Race

pytestmark = pytest.mark.gpu
L = inputs.TRACK_LEN


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _paced(n, seed):
    rng = np.random.default_rng(seed)
    return inputs.pace_params(rng, inputs.competitor_params(rng, n))


def _compare(torch, orc, comp, n_sims, seed, request=0, state=None, stop_after=None):
    announce(f"paced n={comp.shape[0]} sims={n_sims} seed={seed} stop={stop_after} "
             f"state={'yes' if state is not None else 'start'}")
    race = Race(comp, L)
    out = api.mc(race, n_sims, seed, request=request, state=state, stop_after=stop_after,
                 want_orders=True)
    torch.cuda.synchronize()
    oo, ow, os_ = orc.race_sim(comp, L, n_sims, seed, request=request, state=state,
                               stop_after=stop_after, threads=8)
    np.testing.assert_array_equal(out["orders"].cpu().numpy(), oo)
    np.testing.assert_array_equal(out["wins"].cpu().numpy().astype(np.uint64), ow)
    assert int(out["steps"].item()) == os_
    return ow


@pytest.mark.parametrize("n", [1, 3, 8, 15, 16, 18, 20])
def test_paced_mc_matches_oracle(torch, orc, n):
    comp = _paced(n, 300 + n)
    _compare(torch, orc, comp, 1000 + 29 * n, seed=n, request=7)
    st = orc.race_prefix(comp, L, 4, 0x80000000 | n, 0, 900.0)
    _compare(torch, orc, comp, 777, seed=n + 1, request=8, state=st)
    _compare(torch, orc, comp, 500, seed=n + 2, request=9, stop_after=max(1, n // 3))


def test_time_term_changes_the_race_and_zero_does_not(torch, orc):
    comp = _paced(20, 11)
    plain = _compare(torch, orc, comp[:, :5], 4000, seed=3)
    paced = _compare(torch, orc, comp, 4000, seed=3)
    assert not np.array_equal(plain, paced)
    zero = comp.copy()
    zero[:, 5] = 0.0  # tau set, gamma 0: the plain kernel, the plain race
    np.testing.assert_array_equal(_compare(torch, orc, zero, 4000, seed=3), plain)


def test_paced_and_plain_requests_in_one_batch(torch, orc):
    rng = np.random.default_rng(21)
    specs, expect = [], []
    for i in range(40):
        n = int(rng.integers(5, 21))
        comp = inputs.competitor_params(rng, n)
        if i % 2:
            comp = inputs.pace_params(rng, comp)
        st = orc.race_prefix(comp, L, 5, 0x80000000 | i, 0, float(rng.uniform(0, 1500)))
        n_sims = int(rng.integers(50, 600))
        specs.append((Race(comp, L), st, 0, n_sims, i, 0))
        _, w, s = orc.race_sim(comp, L, n_sims, 5, request=i, state=st, want_orders=False,
                               threads=8)
        expect.append((w, s))
    announce("batch of 40 requests, every other one paced")
    wins = torch.zeros((40, 20), dtype=torch.int64, device="cuda")
    probs = torch.zeros((40, 20), dtype=torch.float64, device="cuda")
    steps = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan = BatchPlan(specs, 5, wins, probs, steps, autotune=True)
    plan.launch()
    torch.cuda.synchronize()
    W = wins.cpu().numpy()
    for i, (w, _) in enumerate(expect):
        np.testing.assert_array_equal(W[i, :w.size].astype(np.uint64), w)
    assert int(steps.item()) == sum(s for _, s in expect)


def test_paced_trace_and_prefix(torch, orc):
    for n in (2, 9, 20):
        comp = _paced(n, 50 + n)
        race = Race(comp, L)
        announce(f"paced trace and prefix n={n}")
        g = api.trace(race, 6, 1, 2, 100000)
        t, p, q = api.prefix(race, 6, 1, 2, 1200.0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.cpu().numpy(), orc.race_trace(comp, L, 6, 1, 2, 100000))
        ot, op, oq = orc.race_prefix(comp, L, 6, 1, 2, 1200.0)
        assert int(t.item()) == ot
        np.testing.assert_array_equal(p.cpu().numpy(), op)
        np.testing.assert_array_equal(q.cpu().numpy(), oq)


def test_paced_prefix_batch(torch, orc):
    """The batched in-play state generator with paced and plain races."""
    from paper_2108_02419_amd import _bbe
    rng = np.random.default_rng(33)
    comps, targets = [], []
    for i in range(64):
        comp = inputs.competitor_params(rng, int(rng.integers(2, 21)))
        comps.append(inputs.pace_params(rng, comp) if i % 3 else comp)
        targets.append(float(rng.uniform(0.0, 1800.0)))
    specs = [(Race(c, L), None, 0, 1, 0x80000000 | i, 0) for i, c in enumerate(comps)]
    n = len(specs)
    tick = torch.zeros(n, dtype=torch.int32, device="cuda")
    pos = torch.zeros((n, 20), dtype=torch.float32, device="cuda")
    prev = torch.zeros((n, 20), dtype=torch.float32, device="cuda")
    announce("paced prefix batch of 64")
    _bbe.prefix_batch(specs, np.zeros(n, np.uint32), targets, 9, tick, pos, prev)
    torch.cuda.synchronize()
    T, P, V = tick.cpu().numpy().view(np.uint32), pos.cpu().numpy(), prev.cpu().numpy()
    for i, c in enumerate(comps):
        ot, op, oq = orc.race_prefix(c, L, 9, 0x80000000 | i, 0, targets[i])
        m = c.shape[0]
        assert T[i] == ot
        np.testing.assert_array_equal(P[i, :m], op)
        np.testing.assert_array_equal(V[i, :m], oq)
