"""GPU parity of the batched path (persistent kernel in a captured graph):
per-request win counts, probabilities and competitor-steps equal the CPU
oracle's; batched equals individual calls; graph replays repeat exactly; the
batched in-play state generator equals the oracle's."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from paper_2108_02419_amd import _bbe, api, inputs
from paper_2108_02419_amd._bbe import BatchPlan, Race

pytestmark = pytest.mark.gpu
L = inputs.TRACK_LEN
SEED = 3


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _oracle_states(orc, reqs):
    return [orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0, r.target) for r in reqs]


def _run_plan(torch, specs, seed, autotune=True):
    n = len(specs)
    wins = torch.zeros((n, 20), dtype=torch.int64, device="cuda")
    probs = torch.zeros((n, 20), dtype=torch.float64, device="cuda")
    steps = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan = BatchPlan(specs, seed, wins, probs, steps, autotune=autotune)
    plan.launch()
    torch.cuda.synchronize()
    return plan, wins, probs, steps


def test_batch_matches_oracle(torch, orc):
    reqs = inputs.batch_requests(n_requests=48)
    states = _oracle_states(orc, reqs)
    races = [Race(r.comp, L) for r in reqs]
    rng = np.random.default_rng(7)
    specs, exp_w, exp_s = [], [], 0
    for i, (r, st, race) in enumerate(zip(reqs, states, races)):
        n_sims = int(min(r.n_sims, 700))
        stop = int(rng.choice([0, 1, max(1, r.n // 2)]))
        begin = int(rng.integers(0, 1000))
        specs.append((race, st, begin, n_sims, r.index, stop))
        _, w, s = orc.race_sim(r.comp, L, n_sims, SEED, request=r.index, state=st,
                               sim_begin=begin, stop_after=stop or r.n, want_orders=False,
                               threads=8)
        exp_w.append(w)
        exp_s += s
    announce(f"batch of {len(specs)} requests")
    plan, wins, probs, steps = _run_plan(torch, specs, SEED)
    W = wins.cpu().numpy()
    P = probs.cpu().numpy()
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(W[i, :r.n].astype(np.uint64), exp_w[i])
        assert (W[i, r.n:] == 0).all()
        np.testing.assert_array_equal(P[i, :r.n], orc.win_probs(exp_w[i]))
        assert (P[i, r.n:] == 0).all()
    assert int(steps.item()) == exp_s
    info = plan.info()
    assert info["waves_per_block"] in (1, 2, 4) and info["n_items"] >= len(specs)


def test_batch_equals_individual_calls_and_replays(torch, orc):
    reqs = inputs.batch_requests(n_requests=24)
    states = _oracle_states(orc, reqs)
    races = [Race(r.comp, L) for r in reqs]
    specs = [(race, st, 0, int(min(r.n_sims, 2000)), r.index, 0)
             for r, st, race in zip(reqs, states, races)]
    plan, wins, probs, steps = _run_plan(torch, specs, SEED, autotune=False)
    first_w, first_p, first_s = wins.clone(), probs.clone(), steps.clone()
    for i, (race, st, b, n_sims, req, _) in enumerate(specs):
        out = api.mc(race, n_sims, SEED, request=req, state=st, sim_begin=b)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out["wins"].cpu().numpy(), first_w[i, :race.n].cpu().numpy())
    # replays of the captured graph, with eager work in between
    for k in range(4):
        junk = torch.randn(1 << 20, device="cuda").sum()
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(wins, first_w) and torch.equal(probs, first_p)
        assert torch.equal(steps, first_s), k
        del junk


def test_prefix_batch_matches_oracle(torch, orc):
    reqs = inputs.batch_requests(n_requests=150)
    races = [Race(r.comp, L) for r in reqs]
    specs = [(race, None, 0, 1, r.prefix_request, 0) for r, race in zip(reqs, races)]
    n = len(specs)
    tick = torch.zeros(n, dtype=torch.int32, device="cuda")
    pos = torch.zeros((n, 20), dtype=torch.float32, device="cuda")
    prev = torch.zeros((n, 20), dtype=torch.float32, device="cuda")
    _bbe.prefix_batch(specs, np.zeros(n, np.uint32), [r.target for r in reqs], SEED, tick, pos,
                      prev)
    torch.cuda.synchronize()
    T, Pp, Pv = tick.cpu().numpy().view(np.uint32), pos.cpu().numpy(), prev.cpu().numpy()
    for i, r in enumerate(reqs):
        ot, op, oq = orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0, r.target)
        assert T[i] == ot
        np.testing.assert_array_equal(Pp[i, :r.n], op)
        np.testing.assert_array_equal(Pv[i, :r.n], oq)


def test_full_batch_workload(torch, orc):
    """The 4096-request workload as the benchmark runs it: states from the
    GPU generator, one autotuned plan; every row tallies exactly its
    simulations, and sampled requests equal the oracle."""
    reqs = inputs.batch_requests()
    announce(f"full batch: {len(reqs)} requests, {sum(r.n_sims for r in reqs)} sims")
    races = [Race(r.comp, L) for r in reqs]
    n = len(reqs)
    tick = torch.zeros(n, dtype=torch.int32, device="cuda")
    pos = torch.zeros((n, 20), dtype=torch.float32, device="cuda")
    prev = torch.zeros((n, 20), dtype=torch.float32, device="cuda")
    _bbe.prefix_batch([(race, None, 0, 1, r.prefix_request, 0) for r, race in zip(reqs, races)],
                      np.zeros(n, np.uint32), [r.target for r in reqs], SEED, tick, pos, prev)
    torch.cuda.synchronize()
    T, Pp, Pv = tick.cpu().numpy().view(np.uint32), pos.cpu().numpy(), prev.cpu().numpy()
    assert (T != 0xFFFFFFFF).all()
    states = [(int(T[i]), Pp[i, :r.n].copy(), Pv[i, :r.n].copy()) for i, r in enumerate(reqs)]
    specs = [(race, st, 0, r.n_sims, r.index, 0) for r, st, race in zip(reqs, states, races)]
    plan, wins, probs, steps = _run_plan(torch, specs, SEED)
    W = wins.cpu().numpy()
    np.testing.assert_array_equal(W.sum(axis=1), [r.n_sims for r in reqs])
    rng = np.random.default_rng(1)
    for i in rng.choice(n, 6, replace=False):
        r = reqs[i]
        ost = orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0, r.target)
        assert ost[0] == states[i][0]
        np.testing.assert_array_equal(ost[1], states[i][1])
        _, w, _ = orc.race_sim(r.comp, L, r.n_sims, SEED, request=r.index, state=ost,
                               want_orders=False, threads=8)
        np.testing.assert_array_equal(W[i, :r.n].astype(np.uint64), w)


def test_batch_edge_cases_and_request_table(torch, orc):
    """Single simulations, the start line next to in-play states, n = 1 and
    n = 20 in one batch, the top of the simulation index range; the packed
    request table gives the same plan as the per-request path."""
    rng = np.random.default_rng(21)
    c1 = inputs.competitor_params(rng, 1)
    c20 = inputs.competitor_params(rng, 20)
    c3 = inputs.competitor_params(rng, 3)
    st3 = orc.race_prefix(c3, L, SEED, 0x80000007, 0, 900.0)
    races = [Race(c1, L), Race(c20, L), Race(c3, L), Race(c20, L)]
    specs = [(races[0], None, 0, 1, 5, 0),
             (races[1], None, 7, 65, 6, 1),
             (races[2], st3, 2**32 - 3, 3, 7, 0),
             (races[3], None, 0, 1, 8, 20)]
    announce("batch edge cases")
    plan, wins, probs, steps = _run_plan(torch, specs, SEED)
    W = wins.cpu().numpy()
    exp_s = 0
    for i, (race, st, b, n_sims, req, stop) in enumerate(specs):
        comp = race.comp
        _, w, s = orc.race_sim(comp, L, n_sims, SEED, request=req, state=st, sim_begin=b,
                               stop_after=stop or race.n, want_orders=False)
        np.testing.assert_array_equal(W[i, :race.n].astype(np.uint64), w)
        exp_s += s
    assert int(steps.item()) == exp_s
    # the same requests as one packed table (states as [B, 20] rows)
    tick = np.zeros(4, np.uint32)
    pos = np.zeros((4, 20), np.float32)
    prev = np.zeros((4, 20), np.float32)
    prev[:] = 1.0
    tick[2], pos[2, :3], prev[2, :3] = st3[0], st3[1], st3[2]
    tab = _bbe.RequestTable(races, [1, 65, 3, 1], [5, 6, 7, 8], [0, 1, 0, 20],
                            [0, 7, 2**32 - 3, 0], tick=tick, pos=pos, prev=prev)
    # requests 0, 1, 3 as tick 0 with every position 0: nobody is ahead of
    # anybody, so the previous steps are never read -- the start of the race
    _, wins2, _, steps2 = _run_plan(torch, tab, SEED)
    assert torch.equal(wins, wins2) and torch.equal(steps, steps2)


def test_plan_set_states_equals_fresh_plan(torch, orc):
    """A plan re-pointed at new start states (the in-play serving loop)
    gives exactly what a plan built for those states gives; a rejected
    update leaves the plan as it was."""
    reqs = inputs.batch_requests(n_requests=30)
    races = [Race(r.comp, L) for r in reqs]
    st_a = _oracle_states(orc, reqs)
    specs = [(race, st, 0, int(min(r.n_sims, 400)), r.index, 0)
             for r, st, race in zip(reqs, st_a, races)]
    announce("plan set_states")
    plan, wins, probs, steps = _run_plan(torch, specs, SEED)
    st_b = [orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0,
                            np.float32(r.target + 0.5 * (L - r.target))) for r in reqs]
    B = len(reqs)
    tick = np.array([s[0] for s in st_b], np.uint32)
    pos = np.zeros((B, 20), np.float32)
    prev = np.ones((B, 20), np.float32)
    for i, s in enumerate(st_b):
        pos[i, :len(s[1])], prev[i, :len(s[2])] = s[1], s[2]
    plan.set_states(tick, pos, prev)
    plan.launch()
    torch.cuda.synchronize()
    got_w, got_s = wins.clone(), steps.clone()
    fresh = [(race, st, 0, sp[3], sp[4], 0) for race, st, sp in zip(races, st_b, specs)]
    _, w2, p2, s2 = _run_plan(torch, fresh, SEED)
    assert torch.equal(got_w, w2) and torch.equal(probs, p2) and torch.equal(got_s, s2)
    bad = pos.copy()
    bad[3, 0] = L  # a position on the line is not an in-play state
    with pytest.raises(_bbe.BBEError):
        plan.set_states(tick, bad, prev)
    plan.launch()
    torch.cuda.synchronize()
    assert torch.equal(wins, got_w) and torch.equal(steps, got_s)


_TUNE_CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2108_02419_amd import _bbe, inputs
torch.cuda.set_device(0)
reqs = inputs.batch_requests(n_requests=64)
races = [_bbe.Race(r.comp, inputs.TRACK_LEN) for r in reqs]
specs = [(race, None, 0, int(min(r.n_sims, 1000)), r.index, 1) for r, race in zip(reqs, races)]
wins = torch.zeros((len(specs), 20), dtype=torch.int64, device="cuda")
plan = _bbe.BatchPlan(specs, 5, wins, autotune=True)
plan.launch()
torch.cuda.synchronize()
print(json.dumps(dict(plan.info(), wins=int(wins.sum().item()))))
"""


def test_tuning_cache_file_is_written_and_read(torch, tmp_path):
    """A plan created with autotuning records its launch shape in the JSON
    cache named by BBE_TUNE_CACHE; a fresh process creating a plan of the
    same size class takes the shape from the file (an entry planted with a
    distinctive shape is the one it uses), with the same results."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, BBE_TUNE_CACHE=str(cache))

    def child():
        out = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root], env=env, timeout=180,
                             capture_output=True, text=True, check=True).stdout
        return json.loads(out.strip().splitlines()[-1])

    announce("tuning cache: first process")
    first = child()
    text = cache.read_text()
    data = json.loads(text)
    assert len(data["entries"]) == 1
    e = data["entries"][0]
    assert {"device", "kernels", "size_class", "waves_per_block", "sims_per_item",
            "cu_share"} <= set(e)
    assert (e["waves_per_block"], e["sims_per_item"]) == \
        (first["waves_per_block"], first["sims_per_item"])
    # plant a shape the tuner would be unlikely to pick for this small batch
    planted = dict(e, waves_per_block=1, sims_per_item=192, cu_share=2)
    if (e["waves_per_block"], e["sims_per_item"]) == (1, 192):
        planted["waves_per_block"] = 2
    cache.write_text(json.dumps({"entries": [planted]}).replace("}]", "}\n]")
                     .replace("[{", "[\n  {"))
    announce("tuning cache: second process")
    second = child()
    assert (second["waves_per_block"], second["sims_per_item"]) == \
        (planted["waves_per_block"], planted["sims_per_item"])
    assert second["wins"] == first["wins"]


def test_work_list_cap_lengthens_items(torch, orc):
    """A batch of more than 2^20 generations (two requests of 3.5*10^7
    simulations) is cut into fewer, longer work items; its win counts and
    competitor-steps equal those of bbe_race_sim on each request, bit for
    bit."""
    reqs = inputs.batch_requests(n_requests=40)
    small = [r for r in reqs if r.n <= 6][:2]
    assert len(small) == 2
    races = [Race(r.comp, L) for r in small]
    # late in the race: short simulations
    states = [orc.race_prefix(r.comp, L, SEED, r.prefix_request, 0, np.float32(1900.0))
              for r in small]
    n_sims = 35_000_000
    specs = [(race, st, 0, n_sims, r.index, 1) for r, st, race in zip(small, states, races)]
    announce("work-list cap: 2 x 3.5e7 sims")
    plan, wins, probs, steps = _run_plan(torch, specs, SEED, autotune=False)
    info = plan.info()
    assert info["sims_per_item"] > 64 and info["n_items"] <= (1 << 20)
    total = 0
    for i, (race, st, _, n, req, stop) in enumerate(specs):
        w = torch.zeros(race.n, dtype=torch.int64, device="cuda")
        s = torch.zeros(1, dtype=torch.int64, device="cuda")
        _bbe.race_sim(race, n, SEED, request=req, state=st, stop_after=stop, wins=w, steps=s)
        torch.cuda.synchronize()
        assert torch.equal(wins[i, :race.n], w), i
        total += int(s.item())
    assert int(steps.item()) == total


def test_batch_of_short_tick_races(torch, orc):
    """A batch of races of 0.1-second ticks (the surrogate's second training
    set and query loop): in-play states of the recipe at dt = 0.1, winner-only
    and full-order requests, against the oracle request by request."""
    a = inputs.surrogate_state_block(9000, 10, dict(inputs.CFG_SURROGATE, dt=0.1))
    specs, exp_w, exp_s = [], [], 0
    for i in range(10):
        k = int(a["n"][i])
        comp = a["comp"][i, :k]
        st = orc.race_prefix(comp, L, SEED, int(a["prefix_request"][i]), 0, float(a["target"][i]))
        stop = 1 if i % 3 else k
        specs.append((Race(comp, L), st, 0, 150 + 37 * i, 7000 + i, stop))
        _, w, s = orc.race_sim(comp, L, 150 + 37 * i, SEED, request=7000 + i, state=st,
                               stop_after=stop, want_orders=False, threads=8)
        exp_w.append(w)
        exp_s += s
    announce("batch of 10 requests at 0.1-second ticks")
    plan, wins, probs, steps = _run_plan(torch, specs, SEED, autotune=False)
    W = wins.cpu().numpy()
    for i in range(10):
        k = int(a["n"][i])
        np.testing.assert_array_equal(W[i, :k].astype(np.uint64), exp_w[i], err_msg=f"request {i}")
        assert (W[i, k:] == 0).all()
    assert int(steps.item()) == exp_s
    plan.free()
