"""GPU parity of the in-play path against the oracle (paper Section 3: the
state of a race is its vector of positions, advanced by Eq. 1 tick by tick;
RP(d) bettors answer from their own dry-runs from that state; Section 6:
bettors re-estimating while one real race runs):

- bbe_race_advance: the state after each chunk of ticks, bit for bit
  against the oracle's run of the same simulation, and the 0xFFFFFFFF
  answer exactly when a competitor crosses inside the chunk;
- a batch plan re-pointed with bbe_batch_plan_set_states: win counts and
  competitor-steps equal to the oracle's Monte-Carlo from the new states;
- the query loop end to end on a few rounds: the watched race's states,
  sampled Monte-Carlo answers and the judge bit for bit against the oracle,
  the encoded features bit for bit, the surrogate's answers against the
  float64 reference network;
- the RP(d) bettor loop end to end on a few rounds: every bettor's win
  counts and probabilities from its own dry-runs, the RP views and the
  cheap bettors' views bit for bit against the oracle."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from oracle import bettors as OB
from oracle import mlp as ref
from paper_2108_02419_amd import _bbe, bettors, inputs, query_loop
from paper_2108_02419_amd._bbe import BatchPlan, Race

pytestmark = pytest.mark.gpu
L = inputs.TRACK_LEN
SEED = 9


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _oracle_state_at(orc, comp, seed, request, row, trace):
    """The oracle's state after `row` ticks from the start: the leader's
    position only grows, so running until it reaches its row-`row` value
    stops at exactly that tick."""
    return orc.race_prefix(comp, L, seed, request, 0, np.float32(trace[row].max()))


def _advance(torch, race, seed, request, k, state):
    tick = torch.empty(1, dtype=torch.int32, device="cuda")
    pos = torch.empty(race.n, dtype=torch.float32, device="cuda")
    prev = torch.empty(race.n, dtype=torch.float32, device="cuda")
    _bbe.race_advance(race, seed, request, 0, k, tick, pos, prev, state=state)
    torch.cuda.synchronize()
    return int(tick.item()) & 0xFFFFFFFF, pos.cpu().numpy(), prev.cpu().numpy()


@pytest.mark.parametrize("n", [1, 5, 20])
def test_race_advance_matches_oracle_until_the_line(torch, orc, n):
    """Chunks of 1..40 ticks from the start to the first crossing; each state
    equals the oracle's (tick, positions, previous steps); the chunk that
    contains the first crossing answers 0xFFFFFFFF."""
    rng = np.random.default_rng(n)
    comp = inputs.competitor_params(rng, n)
    comp[:, 4] = rng.uniform(0.0, 6.0, n).astype(np.float32)  # blocking happens
    request = 0xC0000000 + n
    race = Race(comp, L)
    trace = orc.race_trace(comp, L, SEED, request, 0, orc.tick_limit() + 1)
    last = trace.shape[0] - 1  # last tick before the first crossing
    announce(f"race_advance n={n}, {last} ticks before the line")
    state, t = None, 0
    while True:
        k = int(rng.integers(1, 41))
        got = _advance(torch, race, SEED, request, k, state)
        if t + k > last:
            assert got[0] == 0xFFFFFFFF, (t, k, last)
            break
        t += k
        want = _oracle_state_at(orc, comp, SEED, request, t, trace)
        assert got[0] == want[0] == t
        np.testing.assert_array_equal(got[1], want[1])
        np.testing.assert_array_equal(got[2], want[2])
        np.testing.assert_array_equal(got[1], trace[t])
        state = (got[0], got[1], got[2])
    # the last in-play state advanced by exactly the ticks left is still in play
    if last > 0:
        st = _oracle_state_at(orc, comp, SEED, request, last - 1, trace)
        got = _advance(torch, race, SEED, request, 1, st)
        assert got[0] == last
        np.testing.assert_array_equal(got[1], trace[last])
        assert _advance(torch, race, SEED, request, 1, (got[0], got[1], got[2]))[0] == \
            0xFFFFFFFF


def test_set_states_plan_matches_oracle(torch, orc):
    """A plan built on one set of in-play states and re-pointed at another:
    per-request win counts, probabilities and the competitor-step total equal
    the oracle's on the new states, for full orders and for stop_after 1."""
    reqs = inputs.batch_requests(n_requests=24)
    races = [Race(r.comp, L) for r in reqs]
    st_a = [orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0, r.target) for r in reqs]
    rng = np.random.default_rng(3)
    for stop in (0, 1):
        specs = [(race, st, int(rng.integers(0, 500)), int(rng.integers(50, 400)), r.index, stop)
                 for r, st, race in zip(reqs, st_a, races)]
        B = len(specs)
        wins = torch.zeros((B, 20), dtype=torch.int64, device="cuda")
        probs = torch.zeros((B, 20), dtype=torch.float64, device="cuda")
        steps = torch.zeros(1, dtype=torch.int64, device="cuda")
        announce(f"set_states plan stop_after={stop}")
        plan = BatchPlan(specs, SEED, wins, probs, steps)
        plan.launch()
        torch.cuda.synchronize()
        # new states: each race further on (a later leader target), or back
        # at the start for a few requests
        st_b = []
        for i, r in enumerate(reqs):
            if i % 7 == 3:
                st_b.append((0, np.zeros(r.n, np.float32), np.ones(r.n, np.float32)))
            else:
                tgt = np.float32(r.target + rng.uniform(0.1, 0.6) * (L - r.target))
                st_b.append(orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0, tgt))
        tick = np.array([s[0] for s in st_b], np.uint32)
        pos = np.zeros((B, 20), np.float32)
        prev = np.ones((B, 20), np.float32)
        for i, s in enumerate(st_b):
            pos[i, :len(s[1])], prev[i, :len(s[2])] = s[1], s[2]
        plan.set_states(tick, pos, prev)
        plan.launch()
        torch.cuda.synchronize()
        W, P = wins.cpu().numpy(), probs.cpu().numpy()
        total = 0
        for i, ((race, _, begin, n_sims, req, _), r, st) in enumerate(zip(specs, reqs, st_b)):
            state = None if st[0] == 0 else st
            _, w, s = orc.race_sim(r.comp, L, n_sims, SEED, request=req, state=state,
                                   sim_begin=begin, stop_after=stop or r.n, want_orders=False,
                                   threads=8)
            total += s
            np.testing.assert_array_equal(W[i, :r.n].astype(np.uint64), w, err_msg=f"request {i}")
            assert (W[i, r.n:] == 0).all()
            np.testing.assert_array_equal(P[i, :r.n], orc.win_probs(w))
        assert int(steps.item()) == total
        plan.free()


def _slot_to_comp(sp, slot, n):
    out = np.zeros(n)
    for r in range(n):
        out[slot[r]] = sp[r]
    return out


@pytest.mark.parametrize("gate,dt,every", [(-1.0, 1.0, 7), (1e9, 1.0, 7), (-1.0, 0.1, 10)],
                         ids=["fallback", "served", "fallback_dt01"])
def test_query_loop_end_to_end(torch, orc, gate, dt, every):
    """Three rounds, `every` ticks apart, 300 bettors: the watched race, the
    1% audit's Monte-Carlo answers and their pooled estimate, the fallback's
    answers (sampled) and the judge against the oracle bit for bit, the
    surrogate's inputs bit for bit and its answers against the reference
    network.  gate -1 sends every round to the fallback; 1e9 (with an audit
    tolerance of 1) serves every round from the surrogate; dt 0.1 is the
    same race with 0.1-second ticks."""
    cfg = dict(inputs.CFG_QUERY, dt=dt)
    q = inputs.query_race(cfg)
    comp, seed, real = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    params = inputs.surrogate_random(8)
    rounds = []
    announce(f"query loop gate={gate} dt={dt}")
    res = query_loop.run(params, every=every, n_bettors=300, mc_sims=400,
                         fallback_sims=[300, "strict"], judge_sims=3000, gate=gate,
                         audit_tol=1.0, baseline_every=2, max_rounds=3, log=lambda m: None,
                         on_round=rounds.append, cfg=cfg)
    assert res["rounds"] == 3 and len(rounds) == 3
    assert res["flagged_rounds"] == (3 if gate < 0 else 0)
    trace = orc.race_trace(comp, L, seed, real, 0, 40)
    rng = np.random.default_rng(4)
    comp_b = np.zeros((1, 20, 5), np.float32)
    comp_b[0, :n] = comp
    for k, rd in enumerate(rounds):
        tick, pos, prev = rd["state"]
        want = _oracle_state_at(orc, comp, seed, real, every * (k + 1), trace)
        assert tick == want[0] == every * (k + 1)
        np.testing.assert_array_equal(pos, want[1])
        np.testing.assert_array_equal(prev, want[2])
        # the audit: 1% of the bettors, each its own request, pooled
        ask, reqs, mp = rd["ask"], rd["requests"], rd["mc_probs"]
        assert len(ask) == 3 and rd["flagged"] == (gate < 0)
        pooled = np.zeros(n, np.uint64)
        for j in range(len(ask)):
            _, w, _ = orc.race_sim(comp, L, 400, rd["mc_seed"], request=int(reqs[j]),
                                   state=rd["state"], stop_after=1, want_orders=False,
                                   threads=8)
            np.testing.assert_array_equal(mp[j, :n], orc.win_probs(w))
            pooled += w
        np.testing.assert_array_equal(rd["pooled"], orc.win_probs(pooled))
        _, wj, _ = orc.race_sim(comp, L, 3000, rd["judge_seed"], request=rd["judge_request"],
                                state=rd["state"], stop_after=1, want_orders=False, threads=8)
        np.testing.assert_array_equal(rd["judge"], orc.win_probs(wj))
        # surrogate: every bettor sees the same state, encoded as the oracle does
        X, slot = ref.encode(comp_b, [n], pos[None, :], prev[None, :], L, dt)
        want_x = (ref.bf16(X).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
        xs = rd["x"].view(np.uint16)
        assert (xs == want_x[0][None, :]).all()
        assert (rd["slot"] == slot[0][None, :]).all()
        sp = rd["sur_probs"]
        assert (sp == sp[0][None, :]).all()
        _, qref, _ = ref.forward(params.astype(np.float64), ref.bf16(X), [n])
        np.testing.assert_allclose(sp[0], qref[0], atol=2e-3)
        assert abs(rd["entropy"][0] - ref.entropy(qref)[0]) <= 5e-3
        sur_c = _slot_to_comp(sp[0], slot[0], n)
        assert np.isclose(rd["audit_gap"], np.abs(sur_c - rd["pooled"]).max())
        # the fallback (flagged rounds): every bettor its own request; sampled
        if gate < 0:
            fb = rd["fallback"]
            assert fb.shape == (300, n)
            for i in sorted(set(rng.choice(300, 3, replace=False).tolist())):
                _, w, _ = orc.race_sim(comp, L, 300, rd["fallback_seed"],
                                       request=int(rd["fallback_base"] + i), state=rd["state"],
                                       stop_after=1, want_orders=False, threads=8)
                np.testing.assert_array_equal(fb[i], orc.win_probs(w))
        else:
            assert rd["fallback"] is None
        # the loop's own error figures are those of these answers
        pr = res["per_round"][k]
        assert np.isclose(pr["sur_err"], np.abs(sur_c - rd["judge"]).max())
        assert np.isclose(pr["mc_err"], np.abs(mp[:, :n] - rd["judge"][None, :]).max())
        if gate < 0:
            assert np.isclose(pr["answer_err"], np.abs(rd["fallback"] - rd["judge"][None, :]).max())
        else:
            assert pr["answer_err"] == pr["sur_err"]
    assert res["seconds"]["baseline_rounds"] == 2  # rounds 0 and 2
    # both fallback sizes ran in the flagged rounds; the strict one is sized
    # from each round's pooled audit estimate
    first, strict = res["fallbacks"]
    assert first["fallback_sims"] == 300 and strict["fallback_sims"] == "strict"
    if gate < 0:
        want = np.mean([query_loop.strict_sims(rd["pooled"]) for rd in rounds])
        assert first["mean_sims"] == 300 and strict["mean_sims"] == want
        assert first["answer_err"]["max"] == res["answer_err"]["max"]
    else:
        assert first["mean_sims"] is None and strict["fallback_seconds"] == 0.0


def test_rp_bettor_loop_end_to_end(torch, orc):
    """Three rounds, 6 ticks apart, 48 RP(d) bettors (d log-uniform in
    1..40) and 256 cheap bettors: each round's state against the oracle's
    trace of the race; every bettor's win counts (its d dry-runs, request =
    its index, from that state, winner only) and probabilities, the RP
    views and their counts, and the cheap bettors' views at the same tick,
    all bit for bit; the loop's dry-run and competitor-step totals are the
    oracle's."""
    q = inputs.query_race()
    comp, seed, real = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    rounds = []
    announce("RP(d) bettor loop")
    res = bettors.run(n_bettors=48, d_lo=1, d_hi=40, every=6, max_rounds=3, n_cheap=256,
                      report_every=0, log=lambda m: None, on_round=rounds.append)
    assert res["rounds"] == 3 and len(rounds) == 3
    trace = orc.race_trace(comp, L, seed, real, 0, 40)
    kinds, params = inputs.cheap_bettors(n_bettors=256)
    d = rounds[0]["d"]
    assert d.min() >= 1 and d.max() <= 40
    total_steps = 0
    for k, rd in enumerate(rounds):
        tick, pos, prev = rd["state"]
        want = _oracle_state_at(orc, comp, seed, real, 6 * (k + 1), trace)
        assert tick == want[0] == 6 * (k + 1)
        np.testing.assert_array_equal(pos, want[1])
        np.testing.assert_array_equal(prev, want[2])
        W = np.zeros((48, n), np.uint64)
        steps = 0
        for i in range(48):
            _, w, s = orc.race_sim(comp, L, int(d[i]), rd["plan_seed"], request=i,
                                   state=rd["state"], stop_after=1, want_orders=False, threads=8)
            W[i] = w
            steps += s
            np.testing.assert_array_equal(rd["wins"][i, :n].astype(np.uint64), w,
                                          err_msg=f"round {k} bettor {i}")
            np.testing.assert_array_equal(rd["probs"][i, :n], orc.win_probs(w))
        assert (rd["wins"][:, n:] == 0).all()
        assert rd["steps"] == steps
        total_steps += steps
        v, c = OB.rp_views(W, n)
        np.testing.assert_array_equal(rd["rp_views"], v)
        np.testing.assert_array_equal(rd["rp_counts"].astype(np.uint32), c)
        assert rd["row"] == tick
        cv, cc = OB.views(kinds, params, trace, L, 0, inputs.CFG_VIEWS["views_seed"],
                          rd["row"], 1)
        np.testing.assert_array_equal(rd["cheap_views"], cv[0])
        np.testing.assert_array_equal(rd["cheap_counts"].astype(np.uint32), cc[0])
    assert res["dry_runs"] == 3 * int(d.sum())
    assert res["competitor_steps"] == total_steps


def test_query_loop_full_size_sampled(torch, orc):
    """The query loop at the size bench.py times (10^4 bettors, 10^4
    simulations per audited and per fallback answer, a 10^6-simulation
    judge), two rounds with every round handed back: sampled audit and
    fallback answers against the oracle one by one, every bettor's
    features bit for bit, and the surrogate's answer against the reference
    network."""
    q = inputs.query_race()
    comp, seed, real = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    params = inputs.surrogate_random(9)
    rounds = []
    announce("query loop full size, 2 rounds")
    res = query_loop.run(params, every=1, n_bettors=10_000, mc_sims=10_000,
                         fallback_sims=[10_000], judge_sims=1_000_000, gate=-1.0,
                         baseline_every=0, max_rounds=2, log=lambda m: None,
                         on_round=rounds.append)
    assert res["rounds"] == 2 and res["flagged_rounds"] == 2
    rng = np.random.default_rng(7)
    comp_b = np.zeros((1, 20, 5), np.float32)
    comp_b[0, :n] = comp
    for rd in rounds:
        tick, pos, prev = rd["state"]
        assert len(rd["ask"]) == 100
        for j in rng.choice(100, 3, replace=False):
            _, w, _ = orc.race_sim(comp, L, 10_000, rd["mc_seed"], request=int(rd["requests"][j]),
                                   state=rd["state"], stop_after=1, want_orders=False,
                                   threads=8)
            np.testing.assert_array_equal(rd["mc_probs"][j, :n], orc.win_probs(w))
        fb = rd["fallback"]
        assert fb.shape == (10_000, n)
        for i in rng.choice(10_000, 3, replace=False):
            _, w, _ = orc.race_sim(comp, L, 10_000, rd["fallback_seed"],
                                   request=int(rd["fallback_base"] + i), state=rd["state"],
                                   stop_after=1, want_orders=False, threads=8)
            np.testing.assert_array_equal(fb[i], orc.win_probs(w))
        X, slot = ref.encode(comp_b, [n], pos[None, :], prev[None, :], L, inputs.CFG_QUERY["dt"])
        want_x = (ref.bf16(X).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
        assert (rd["x"].view(np.uint16) == want_x[0][None, :]).all()
        _, qref, _ = ref.forward(params.astype(np.float64), ref.bf16(X), [n])
        np.testing.assert_allclose(rd["sur_probs"][0], qref[0], atol=2e-3)


def test_rp_bettor_loop_full_size_sampled(torch, orc):
    """The RP(d) bettor loop at the size bench.py times (10^4 bettors with d
    log-uniform in 1..200, 10^5 cheap bettors), two rounds: sampled bettors'
    win counts and views, and sampled cheap bettors' views, against the
    oracle one by one; the RP view counts against the views."""
    q = inputs.query_race()
    comp, seed, real = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    rounds = []
    announce("RP(d) bettor loop full size, 2 rounds")
    res = bettors.run(n_bettors=10_000, d_lo=1, d_hi=200, every=1, max_rounds=2,
                      n_cheap=100_000, report_every=0, log=lambda m: None,
                      on_round=rounds.append)
    assert res["rounds"] == 2
    trace = orc.race_trace(comp, L, seed, real, 0, 10)
    kinds, params = inputs.cheap_bettors(n_bettors=100_000)
    rng = np.random.default_rng(8)
    for rd in rounds:
        d = rd["d"]
        for i in rng.choice(10_000, 4, replace=False):
            _, w, _ = orc.race_sim(comp, L, int(d[i]), rd["plan_seed"], request=int(i),
                                   state=rd["state"], stop_after=1, want_orders=False, threads=8)
            np.testing.assert_array_equal(rd["wins"][i, :n].astype(np.uint64), w)
            v, _ = OB.rp_views(w[None, :], n)
            assert rd["rp_views"][i] == v[0]
        np.testing.assert_array_equal(np.bincount(rd["rp_views"], minlength=n), rd["rp_counts"])
        for b in rng.choice(100_000, 20, replace=False):
            want = OB.view(int(kinds[b]), float(params[b]), trace, rd["row"], L, 0, int(b),
                           inputs.CFG_VIEWS["views_seed"])
            assert rd["cheap_views"][b] == want, b
