"""In-play query loop: one race watched by many bettors who re-estimate the
win probabilities at a fixed period (paper Section 3: RP(d) bettors; Section
6: every bettor updating its private estimate once per second, one real race
plus the bettors' dry-runs).

Per round: the real race advances `every` ticks (its own random stream);
all bettors query the surrogate on the new state; a sample of the queries,
plus every query whose surrogate entropy exceeds a threshold, is answered by
Monte-Carlo instead (each bettor its own simulations, as its own request);
a high-sample Monte-Carlo judge measures the error of both.  Orchestration
only -- every computation runs in the library's kernels.

    python -m paper_2108_02419_amd.query_loop --params gpurun_out/surrogate/params.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import _bbe, inputs

L = inputs.TRACK_LEN


def _plan_probs(specs, seed, n_rows):
    wins = torch.zeros((n_rows, 20), dtype=torch.int64, device="cuda")
    probs = torch.zeros((n_rows, 20), dtype=torch.float64, device="cuda")
    plan = _bbe.BatchPlan(specs, seed, wins, probs, None, autotune=True)
    return plan, probs


def run(params, every=1, n_bettors=10_000, audit_frac=0.01, mc_sims=10_000,
        judge_sims=1_000_000, entropy_frac=0.95, max_rounds=None, log=print):
    cfg = inputs.CFG_QUERY
    q = inputs.query_race(cfg)
    comp, seed, real_req = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    race = _bbe.Race(comp, L)
    net = _bbe.Mlp(params, max_batch=8)
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)

    comp_b = torch.tensor(np.broadcast_to(np.pad(comp, ((0, 20 - n), (0, 0))),
                                          (n_bettors, 20, 5)).copy(), device=dev)
    n_b = torch.full((n_bettors,), n, dtype=torch.int32, device=dev)
    x = torch.empty((n_bettors, 160), dtype=torch.int16, device=dev)
    slot = torch.empty((n_bettors, 20), dtype=torch.int32, device=dev)
    sprobs = torch.empty((n_bettors, 20), dtype=torch.float32, device=dev)
    sent = torch.empty(n_bettors, dtype=torch.float32, device=dev)
    tick_t = torch.empty(1, dtype=torch.int32, device=dev)
    pos_t = torch.empty(n, dtype=torch.float32, device=dev)
    prev_t = torch.empty(n, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    thr = entropy_frac * math.log(n)

    state = None
    rounds = []
    sur_s = mc_s = 0.0
    sur_q = mc_q = 0
    while max_rounds is None or len(rounds) < max_rounds:
        _bbe.race_advance(race, seed, real_req, 0, every, tick_t, pos_t, prev_t, state=state)
        torch.cuda.synchronize()
        tick = int(tick_t.item()) & 0xFFFFFFFF
        if tick == 0xFFFFFFFF:
            break  # the real race reached its first finisher
        pos, prev = pos_t.cpu().numpy().copy(), prev_t.cpu().numpy().copy()
        state = (tick, pos, prev)

        # every bettor asks the surrogate (no deduplication of equal states)
        pos_b = torch.zeros((n_bettors, 20), dtype=torch.float32, device=dev)
        prev_b = torch.zeros((n_bettors, 20), dtype=torch.float32, device=dev)
        pos_b[:, :n] = pos_t
        prev_b[:, :n] = prev_t
        torch.cuda.synchronize()
        e0.record()
        _bbe.encode_states(comp_b, n_b, pos_b, prev_b, L, cfg["dt"], x, slot)
        net.forward(x, n_b, sprobs, sent)
        e1.record()
        torch.cuda.synchronize()
        t_sur = e0.elapsed_time(e1) / 1e3
        sur_s += t_sur
        sur_q += n_bettors

        ent = sent.cpu().numpy()
        flagged = np.nonzero(ent > thr)[0]
        audit = rng.choice(n_bettors, max(1, int(round(audit_frac * n_bettors))), replace=False)
        ask_mc = np.union1d(flagged, audit)
        base = (len(rounds) * n_bettors) & 0x3FFFFFFF
        specs = [(race, state, 0, mc_sims, base + int(b), 1) for b in ask_mc]
        plan, mprobs = _plan_probs(specs, seed + 1, len(specs))
        e0.record()
        plan.launch()
        e1.record()
        torch.cuda.synchronize()
        t_mc = e0.elapsed_time(e1) / 1e3
        mc_s += t_mc
        mc_q += len(specs)
        plan.free()

        jplan, jprobs = _plan_probs([(race, state, 0, judge_sims, 0x40000000 | len(rounds), 1)],
                                    seed + 2, 1)
        jplan.launch()
        torch.cuda.synchronize()
        jplan.free()
        judge = jprobs.cpu().numpy()[0, :n]
        # surrogate answers are in slot order; map them back to competitors
        sl = slot.cpu().numpy()[0]
        sp = sprobs.cpu().numpy()[0]
        sur_c = np.zeros(n)
        for r in range(n):
            sur_c[sl[r]] = sp[r]
        mc_c = mprobs.cpu().numpy()[:, :n]
        rounds.append(dict(tick=tick, leader=float(pos.max()), entropy=float(ent[0]),
                           flagged=int(len(flagged)), mc_queries=len(specs),
                           sur_err=float(np.abs(sur_c - judge).max()),
                           mc_err=float(np.abs(mc_c - judge[None, :]).max()),
                           t_sur=t_sur, t_mc=t_mc))
        if len(rounds) % 25 == 0:
            r = rounds[-1]
            log(f"round {len(rounds)} tick {tick} leader {r['leader']:.0f} sur_err "
                f"{r['sur_err']:.4f} mc_err {r['mc_err']:.4f} flagged {r['flagged']}")
    sur_err = np.array([r["sur_err"] for r in rounds])
    mc_err = np.array([r["mc_err"] for r in rounds])
    return dict(rounds=len(rounds), bettors=n_bettors, every=every, mc_sims=mc_sims,
                judge_sims=judge_sims, entropy_threshold=thr,
                surrogate_queries_per_s=sur_q / sur_s, mc_queries_per_s=mc_q / mc_s,
                speedup=(sur_q / sur_s) / (mc_q / mc_s),
                surrogate_err=dict(max=float(sur_err.max()), mean=float(sur_err.mean()),
                                   p99=float(np.quantile(sur_err, 0.99))),
                mc_err=dict(max=float(mc_err.max()), mean=float(mc_err.mean())),
                flagged_rounds=int(sum(r["flagged"] > 0 for r in rounds)),
                per_round=rounds)


def main():
    ap = argparse.ArgumentParser(description="in-play query loop")
    ap.add_argument("--params", required=True, help="trained surrogate parameters (.npy)")
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--bettors", type=int, default=10_000)
    ap.add_argument("--judge-sims", type=int, default=1_000_000)
    ap.add_argument("--max-rounds", type=int, default=None)
    ap.add_argument("--out", default="gpurun_out/query_loop.json")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    params = np.load(args.params)
    t0 = time.perf_counter()
    res = run(params, every=args.every, n_bettors=args.bettors, judge_sims=args.judge_sims,
              max_rounds=args.max_rounds, log=lambda m: print(f"[query] {m}", flush=True))
    res["wall_s"] = time.perf_counter() - t0
    summary = {k: v for k, v in res.items() if k != "per_round"}
    print(json.dumps(summary), flush=True)
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
