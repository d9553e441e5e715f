"""RP(d) bettors in play: every bettor re-estimates the win probabilities of
the race in play once per tick (once per second) from its own d dry-runs
(paper Section 3: the RP(d) bettor; Section 6: B bettors of d = 50 updating
once per second need 15000 x B dry-runs for a five-minute race).  One batch
plan serves all bettors for the whole race: each round only the start state
of their requests changes (bbe_batch_plan_set_states), and the plan's graph
is launched again.  Alongside them a population of cheap bettors (Section
5: LinEx, LW, UD, ZI) re-forms its views every round from the trace of the
race in play, and each RP(d) bettor's view is the competitor that won most
of its dry-runs.  Orchestration only -- every simulation and every view
runs in the library's kernels.

    python -m paper_2108_02419_amd.bettors --bettors 10000 --d-lo 1 --d-hi 200 --cheap 100000
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import _bbe, api, inputs

L = inputs.TRACK_LEN


def bettor_sims(n_bettors: int, d_lo: int, d_hi: int, seed: int) -> np.ndarray:
    """d per bettor, log-uniform integers in [d_lo, d_hi] (seeded)."""
    rng = np.random.default_rng([seed, 0xBE77])
    u = rng.uniform(math.log(d_lo), math.log(d_hi + 1), size=n_bettors)
    return np.minimum(np.floor(np.exp(u)).astype(np.int64), d_hi).clip(d_lo)


KIND_NAMES = ("ZI", "LW", "UD", "LinEx")


def run(n_bettors=10_000, d_lo=1, d_hi=200, every=1, max_rounds=None, judge_every=0,
        judge_sims=1_000_000, n_cheap=0, report_every=25, log=print, on_round=None):
    """Steps the query race `every` ticks at a time until its first
    finisher; each round, every RP(d) bettor runs its d dry-runs (winner
    only, its own request id = its index, plan seed = race seed + 3) from
    the state reached, and takes the competitor that won most of them as
    its view; `n_cheap` cheap bettors re-form their views from the race's
    trace at the same tick.  `judge_every` > 0 measures the RP(d)
    estimates' error against a `judge_sims` Monte-Carlo run every that
    many rounds.

    `on_round`, when given, receives each round's host copies: the state
    (tick, pos, prev), the bettors' d, the plan seed, their win counts and
    probabilities ([bettors, 20]), the RP views and view counts and, with
    cheap bettors, the trace row and their views and view counts."""
    cfg = inputs.CFG_QUERY
    q = inputs.query_race(cfg)
    comp, seed, real_req = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    race = _bbe.Race(comp, L)
    dev = torch.device("cuda")
    d = bettor_sims(n_bettors, d_lo, d_hi, seed)
    tick_t = torch.empty(1, dtype=torch.int32, device=dev)
    pos_t = torch.empty(n, dtype=torch.float32, device=dev)
    prev_t = torch.empty(n, dtype=torch.float32, device=dev)

    def advance(state):
        _bbe.race_advance(race, seed, real_req, 0, every, tick_t, pos_t, prev_t, state=state)
        torch.cuda.synchronize()
        tick = int(tick_t.item()) & 0xFFFFFFFF
        if tick == 0xFFFFFFFF:
            return None
        return (tick, pos_t.cpu().numpy().copy(), prev_t.cpu().numpy().copy())

    state = advance(None)
    # the race in play, tick by tick, for the cheap bettors; its rows are the
    # states the loop below reaches with bbe_race_advance
    trace = api.trace(race, seed, real_req, 0, 1 << 16)
    n_rows = int(trace.shape[0])
    if not np.array_equal(trace[every].cpu().numpy(), state[1]):
        raise RuntimeError("race trace and advanced state disagree")
    winner = int(torch.argmax(api.mc(race, 1, seed, request=real_req, stop_after=1)["wins"]))
    cheap = None
    if n_cheap:
        kinds, params = inputs.cheap_bettors(n_bettors=n_cheap)
        cheap = _bbe.Bettors(kinds, params)
        cheap_views = torch.empty((1, n_cheap), dtype=torch.uint8, device=dev)
        cheap_counts = torch.empty((1, n), dtype=torch.int32, device=dev)
    rp_views = torch.empty(n_bettors, dtype=torch.uint8, device=dev)
    rp_counts = torch.empty(n, dtype=torch.int32, device=dev)
    backing = {}
    wins = torch.zeros((n_bettors, 20), dtype=torch.int64, device=dev)
    probs = torch.zeros((n_bettors, 20), dtype=torch.float64, device=dev)
    steps = torch.zeros(1, dtype=torch.int64, device=dev)
    t_setup = time.perf_counter()
    tab = _bbe.RequestTable([race] * n_bettors, d, np.arange(n_bettors), 1,
                            tick=np.full(n_bettors, state[0], np.uint32),
                            pos=np.broadcast_to(state[1], (n_bettors, n)),
                            prev=np.broadcast_to(state[2], (n_bettors, n)))
    plan = _bbe.BatchPlan(tab, seed + 3, wins, probs, steps, autotune=True)
    setup_s = time.perf_counter() - t_setup
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    gpu_s = host_s = views_s = 0.0
    rounds, dry_runs, csteps = 0, 0, 0
    judged = []
    while state is not None and (max_rounds is None or rounds < max_rounds):
        h0 = time.perf_counter()
        if rounds:
            plan.set_states(np.full(n_bettors, state[0], np.uint32),
                            np.broadcast_to(state[1], (n_bettors, n)),
                            np.broadcast_to(state[2], (n_bettors, n)))
        host_s += time.perf_counter() - h0
        e0.record()
        plan.launch()
        e1.record()
        row = (rounds + 1) * every
        _bbe.rp_views(wins, n, views=rp_views, counts=rp_counts)
        if cheap is not None and row < n_rows:
            cheap.views(trace, n_rows, L, 0, inputs.CFG_VIEWS["views_seed"], row, 1,
                        views=cheap_views, counts=cheap_counts)
        e2.record()
        torch.cuda.synchronize()
        gpu_s += e0.elapsed_time(e1) / 1e3
        views_s += e1.elapsed_time(e2) / 1e3
        if report_every and rounds % report_every == 0:
            frac = {"RP": float((rp_views == winner).float().mean())}
            if cheap is not None and row < n_rows:
                cv = cheap_views[0].cpu().numpy()
                for k, name in enumerate(KIND_NAMES):
                    frac[name] = float((cv[kinds == k] == winner).mean())
            backing[int(state[0])] = frac
        csteps += int(steps.item())
        dry_runs += int(d.sum())
        if on_round is not None:
            rd = dict(round=rounds, state=state, d=d, plan_seed=seed + 3,
                      wins=wins.cpu().numpy(), probs=probs.cpu().numpy(),
                      rp_views=rp_views.cpu().numpy(), rp_counts=rp_counts.cpu().numpy(),
                      steps=int(steps.item()))
            if cheap is not None and row < n_rows:
                rd.update(row=row, cheap_views=cheap_views[0].cpu().numpy(),
                          cheap_counts=cheap_counts[0].cpu().numpy())
            on_round(rd)
        rounds += 1
        if judge_every and rounds % judge_every == 0:
            judged.append(_judge(race, state, n, probs, d, judge_sims, seed, rounds))
        state = advance(state)
    res = dict(bettors=n_bettors, d_lo=d_lo, d_hi=d_hi, d_mean=float(d.mean()), rounds=rounds,
               dry_runs=dry_runs, competitor_steps=csteps, gpu_seconds=gpu_s,
               host_seconds_set_states=host_s, plan_setup_seconds=setup_s,
               dry_runs_per_s=dry_runs / gpu_s, bettor_updates_per_s=rounds * n_bettors / gpu_s,
               gpu_ms_per_round=1e3 * gpu_s / max(1, rounds), plan=plan.info(),
               cheap_bettors=n_cheap, views_gpu_ms_per_round=1e3 * views_s / max(1, rounds),
               winner=winner, backing_winner_by_tick=backing)
    if judged:
        res["rp_error_by_d"] = _merge(judged)
    plan.free()
    return res


def _judge(race, state, n, probs, d, judge_sims, seed, rnd):
    """Max abs error of each bettor's estimate against a judge run."""
    jt = _bbe.RequestTable([race], judge_sims, [0x40000000 | rnd], 1,
                           tick=np.array([state[0]], np.uint32), pos=state[1][None, :],
                           prev=state[2][None, :])
    jw = torch.zeros((1, 20), dtype=torch.int64, device="cuda")
    jp = torch.zeros((1, 20), dtype=torch.float64, device="cuda")
    jplan = _bbe.BatchPlan(jt, seed + 4, jw, jp, None, autotune=False)
    jplan.launch()
    torch.cuda.synchronize()
    judge = jp.cpu().numpy()[0, :n]
    jplan.free()
    err = np.abs(probs.cpu().numpy()[:, :n] - judge[None, :]).max(axis=1)
    return d, err


def _merge(judged):
    d = np.concatenate([x[0] for x in judged])
    e = np.concatenate([x[1] for x in judged])
    out = {}
    for lo, hi in [(1, 4), (4, 16), (16, 64), (64, 256), (256, 1 << 30)]:
        m = (d >= lo) & (d < hi)
        if m.any():
            out[f"d_{lo}_{hi if hi < (1 << 30) else 'inf'}"] = dict(
                bettor_rounds=int(m.sum()), mean_max_abs=float(e[m].mean()),
                p90_max_abs=float(np.quantile(e[m], 0.9)))
    return out


def main():
    ap = argparse.ArgumentParser(description="RP(d) bettors updating every tick of a race")
    ap.add_argument("--bettors", type=int, default=10_000)
    ap.add_argument("--d-lo", type=int, default=1)
    ap.add_argument("--d-hi", type=int, default=200)
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--max-rounds", type=int, default=None)
    ap.add_argument("--judge-every", type=int, default=25)
    ap.add_argument("--cheap", type=int, default=100_000, help="LinEx/LW/UD/ZI bettors")
    ap.add_argument("--out", default="bbe_out/bettors.json")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    res = run(args.bettors, args.d_lo, args.d_hi, args.every, args.max_rounds,
              judge_every=args.judge_every, n_cheap=args.cheap, log=lambda m: print(f"[bettors] {m}", flush=True))
    res["wall_s"] = time.perf_counter() - t0
    print(json.dumps(res), flush=True)
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
