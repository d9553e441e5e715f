"""One fault-injection case of tests/test_gpu_faults.py, run in a process of
its own: the library reads BBE_FAULT_INJECT once per process, so each case
starts fresh.  Prints one JSON line: the outcome of every call the case
makes ([code, message] per attempt; code 0 = success) and the checks of the
results computed after the failures.

    BBE_FAULT_INJECT="device:1,4,8" python tests/fault_cases.py race_sim
"""
import json
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2108_02419_amd import _bbe, inputs  # noqa: E402

L = inputs.TRACK_LEN


def attempt(fn):
    """[0, ""] if fn() returns, [code, message] if it raises BBEError."""
    try:
        fn()
        torch.cuda.synchronize()
        return [0, ""]
    except _bbe.BBEError as e:
        torch.cuda.synchronize()
        return [e.code, str(e)]


def race_sim_case():
    comp = inputs.competitor_params(np.random.default_rng(1), 5)
    race = _bbe.Race(comp, L)
    wins = torch.zeros(5, dtype=torch.int64, device="cuda")
    steps = torch.zeros(1, dtype=torch.int64, device="cuda")
    probs = torch.zeros(5, dtype=torch.float64, device="cuda")
    run = lambda: _bbe.race_sim(race, 3000, 7, wins=wins, steps=steps)  # noqa: E731
    out = [attempt(run), attempt(run), attempt(run)]
    w1 = wins.cpu().numpy().copy()
    out.append(attempt(lambda: _bbe.win_probs(wins, probs)))
    out.append(attempt(lambda: _bbe.win_probs(wins, probs)))
    out.append(attempt(run))
    checks = {"wins_repeat": bool((wins.cpu().numpy() == w1).all()),
              "wins_total": int(w1.sum()) == 3000,
              "probs": bool(np.allclose(probs.cpu().numpy(), w1 / 3000.0, rtol=0, atol=0))}
    return out, checks


def _plan_specs():
    reqs = inputs.batch_requests(n_requests=6)
    races = [_bbe.Race(r.comp, L) for r in reqs]
    return [(race, None, 0, 200 + 50 * i, r.index, 0) for i, (r, race) in
            enumerate(zip(reqs, races))]


def plan_case():
    specs = _plan_specs()
    wins = torch.zeros((6, 20), dtype=torch.int64, device="cuda")
    out, plans = [], []

    def create():
        plans.append(_bbe.BatchPlan(specs, 3, wins, autotune=False))

    for _ in range(6):
        r = attempt(create)
        out.append(r)
        if r[0] == 0:
            break
    plan = plans[-1] if plans else None
    if plan is not None:
        out.append(attempt(plan.launch))
        out.append(attempt(plan.launch))
    W = wins.cpu().numpy()
    # each request alone through bbe_race_sim: the same win counts
    same = True
    for i, (race, _, begin, n_sims, req, _) in enumerate(specs):
        w = torch.zeros(race.n, dtype=torch.int64, device="cuda")
        _bbe.race_sim(race, n_sims, 3, request=req, sim_begin=begin, wins=w)
        torch.cuda.synchronize()
        same &= bool((w.cpu().numpy() == W[i, :race.n]).all())
    if plan is not None:
        plan.free()
    return out, {"plan_created": plan is not None, "wins_equal_individual": same}


def mlp_case():
    params = inputs.surrogate_random(3)
    x = torch.tensor(np.random.default_rng(0).integers(0, 1 << 14, (8, 160)).astype(np.int16),
                     device="cuda")
    nv = torch.full((8,), 20, dtype=torch.int32, device="cuda")
    probs = torch.zeros((8, 20), dtype=torch.float32, device="cuda")
    nets, out = [], []
    for _ in range(4):
        r = attempt(lambda: nets.append(_bbe.Mlp(params, max_batch=8)))
        out.append(r)
        if r[0] == 0:
            break
    net = nets[-1]
    out.append(attempt(lambda: net.forward(x, nv, probs)))
    out.append(attempt(lambda: net.forward(x, nv, probs)))
    ref = torch.zeros_like(probs)
    _bbe.Mlp(params, max_batch=8).forward(x, nv, ref)
    torch.cuda.synchronize()
    return out, {"forward_equal": bool(torch.equal(probs, ref)),
                 "params_equal": bool((net.params() == params.astype(np.float32)).all())}


def bettors_case():
    kinds, params = inputs.cheap_bettors(n_bettors=300)
    rng = np.random.default_rng(2)
    tr = torch.tensor(np.cumsum(rng.uniform(1.0, 3.0, (40, 6)), axis=0).astype(np.float32),
                      device="cuda")
    objs, out = [], []
    for _ in range(4):
        r = attempt(lambda: objs.append(_bbe.Bettors(kinds, params)))
        out.append(r)
        if r[0] == 0:
            break
    b = objs[-1]
    views = torch.zeros((40, 300), dtype=torch.uint8, device="cuda")
    run = lambda: b.views(tr, 40, 200.0, 0, 5, 0, 40, views=views)  # noqa: E731
    out.append(attempt(run))
    out.append(attempt(run))
    ref = torch.zeros_like(views)
    _bbe.Bettors(kinds, params).views(tr, 40, 200.0, 0, 5, 0, 40, views=ref)
    torch.cuda.synchronize()
    return out, {"views_equal": bool(torch.equal(views, ref))}


def _prefix_inputs():
    reqs = inputs.batch_requests(n_requests=10)
    races = [_bbe.Race(r.comp, L) for r in reqs]
    specs = [(race, None, 0, 1, r.prefix_request, 0) for r, race in zip(reqs, races)]
    return specs, np.zeros(10, np.uint32), np.array([r.target for r in reqs], np.float32)


def prefix_case(noalloc: bool):
    specs, sims, targets = _prefix_inputs()
    outs = [(torch.zeros(10, dtype=torch.int32, device="cuda"),
             torch.zeros((10, 20), dtype=torch.float32, device="cuda"),
             torch.zeros((10, 20), dtype=torch.float32, device="cuda")) for _ in range(2)]
    fn = _bbe.prefix_batch_noalloc if noalloc else _bbe.prefix_batch
    out = [attempt(lambda: fn(specs, sims, targets, 9, *outs[0])) for _ in range(3)]
    # the reference: bbe_prefix_batch, tried again if an injected fault hits it
    for _ in range(2):
        r = attempt(lambda: _bbe.prefix_batch(specs, sims, targets, 9, *outs[1]))
        out.append(r)
        if r[0] == 0:
            break
    same = all(torch.equal(a, b) for a, b in zip(outs[0], outs[1]))
    return out, {"states_equal": same}


CASES = {"race_sim": race_sim_case, "plan": plan_case, "mlp": mlp_case,
         "bettors": bettors_case, "prefix": lambda: prefix_case(False),
         "prefix_noalloc": lambda: prefix_case(True)}

if __name__ == "__main__":
    torch.cuda.set_device(0)
    outcomes, checks = CASES[sys.argv[1]]()
    print(json.dumps({"outcomes": outcomes, "checks": checks}), flush=True)
