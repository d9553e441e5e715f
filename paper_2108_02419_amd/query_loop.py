"""In-play query loop: one race watched by many bettors who re-estimate the
win probabilities at a fixed period (paper Section 3: RP(d) bettors; Section
6: every bettor updating its private estimate once per second, one real race
plus the bettors' dry-runs).

Per round: the real race advances `every` ticks (its own random stream);
all bettors query the surrogate on the new state; when the surrogate's
entropy exceeds a gate every bettor's query goes to Monte-Carlo instead
(each bettor its own simulations, as its own request), otherwise a random
audit sample is also answered by Monte-Carlo; a high-sample Monte-Carlo
judge measures the error of both.  Orchestration only -- every computation
runs in the library's kernels.

    python -m paper_2108_02419_amd.query_loop --params bbe_out/surrogate/params.npy
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


def _mc_answers(race, state, n, n_queries, requests, mc_sims, seed):
    """Monte-Carlo answers for `n_queries` bettors on one state (each bettor
    its own request); returns (plan, probs [n_queries, 20])."""
    tick, pos, prev = state
    tab = _bbe.RequestTable([race] * n_queries, mc_sims, requests, 1,
                            tick=np.full(n_queries, tick, np.uint32),
                            pos=np.broadcast_to(pos, (n_queries, n)),
                            prev=np.broadcast_to(prev, (n_queries, n)))
    wins = torch.zeros((n_queries, 20), dtype=torch.int64, device="cuda")
    probs = torch.zeros((n_queries, 20), dtype=torch.float64, device="cuda")
    plan = _bbe.BatchPlan(tab, seed, wins, probs, None, autotune=True)
    return plan, probs


def run(params, every=1, n_bettors=10_000, audit_frac=0.01, mc_sims=10_000,
        judge_sims=1_000_000, gate=None, max_rounds=None, log=print, on_round=None):
    """Steps the real race and answers every bettor each round.  A round's
    state goes to Monte-Carlo for every bettor when the surrogate's entropy
    exceeds `gate` (default 0.95 ln n); otherwise the surrogate answers and
    a random `audit_frac` of the bettors is also answered by Monte-Carlo.
    `on_round`, when given, receives each round's host copies: the state
    (tick, pos, prev), the asked bettors and their request ids, the
    Monte-Carlo answers (float64 [asked, 20], competitor order), the judge's
    answer, the encoded features and slot map of every bettor, and the
    surrogate's answers (float32 [bettors, 20], slot order)."""
    cfg = inputs.CFG_QUERY
    q = inputs.query_race(cfg)
    comp, seed, real_req = q["comp"], q["seed"], q["real_request"]
    n = comp.shape[0]
    race = _bbe.Race(comp, L)
    net = _bbe.Mlp(params, max_batch=8)
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)
    thr = 0.95 * math.log(n) if gate is None else float(gate)

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
        flagged = bool(ent[0] > thr)
        ask = np.arange(n_bettors) if flagged else np.sort(
            rng.choice(n_bettors, max(1, int(round(audit_frac * n_bettors))), replace=False))
        base = (len(rounds) * n_bettors) & 0x3FFFFFFF
        plan, mprobs = _mc_answers(race, state, n, len(ask), base + ask, mc_sims, seed + 1)
        e0.record()
        plan.launch()
        e1.record()
        torch.cuda.synchronize()
        t_mc = e0.elapsed_time(e1) / 1e3
        mc_s += t_mc
        mc_q += len(ask)
        plan.free()

        jplan, jprobs = _mc_answers(race, state, n, 1, [0x40000000 | len(rounds)], judge_sims,
                                    seed + 2)
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
        sur_err = float(np.abs(sur_c - judge).max())
        mc_err = float(np.abs(mc_c - judge[None, :]).max())
        if on_round is not None:
            on_round(dict(round=len(rounds), state=state, ask=ask, requests=base + ask,
                          mc_seed=seed + 1, judge_request=0x40000000 | len(rounds),
                          judge_seed=seed + 2, mc_probs=mprobs.cpu().numpy(), judge=judge,
                          x=x.cpu().numpy(), slot=slot.cpu().numpy(),
                          sur_probs=sprobs.cpu().numpy(), entropy=ent, flagged=flagged))
        rounds.append(dict(tick=tick, leader=float(pos.max()), entropy=float(ent[0]),
                           flagged=flagged, mc_queries=int(len(ask)), sur_err=sur_err,
                           mc_err=mc_err, answer_err=mc_err if flagged else sur_err,
                           t_sur=t_sur, t_mc=t_mc))
        if len(rounds) % 25 == 0:
            r = rounds[-1]
            log(f"round {len(rounds)} tick {tick} leader {r['leader']:.0f} sur_err "
                f"{r['sur_err']:.4f} mc_err {r['mc_err']:.4f} flagged {r['flagged']}")
    sur_err = np.array([r["sur_err"] for r in rounds])
    mc_err = np.array([r["mc_err"] for r in rounds])
    ans_err = np.array([r["answer_err"] for r in rounds])
    n_flag = int(sum(r["flagged"] for r in rounds))
    total_q = len(rounds) * n_bettors
    mc_qps = mc_q / mc_s
    sys_qps = total_q / (sur_s + mc_s)
    return dict(rounds=len(rounds), bettors=n_bettors, every=every, mc_sims=mc_sims,
                judge_sims=judge_sims, entropy_threshold=thr, audit_frac=audit_frac,
                surrogate_queries_per_s=sur_q / sur_s, mc_queries_per_s=mc_qps,
                speedup=(sur_q / sur_s) / mc_qps,
                system_queries_per_s=sys_qps, system_speedup=sys_qps / mc_qps,
                flagged_rounds=n_flag, served_frac=1.0 - n_flag / max(1, len(rounds)),
                surrogate_err=dict(max=float(sur_err.max()), mean=float(sur_err.mean()),
                                   p99=float(np.quantile(sur_err, 0.99)),
                                   p999=float(np.quantile(sur_err, 0.999))),
                answer_err=dict(max=float(ans_err.max()), mean=float(ans_err.mean()),
                                p999=float(np.quantile(ans_err, 0.999))),
                mc_err=dict(max=float(mc_err.max()), mean=float(mc_err.mean()),
                            p999=float(np.quantile(mc_err, 0.999))),
                per_round=rounds)


def main():
    ap = argparse.ArgumentParser(description="in-play query loop")
    ap.add_argument("--params", required=True, help="trained surrogate parameters (.npy)")
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--bettors", type=int, default=10_000)
    ap.add_argument("--judge-sims", type=int, default=1_000_000)
    ap.add_argument("--max-rounds", type=int, default=None)
    ap.add_argument("--gate", default=None,
                    help="surrogate entropy above which a state goes to Monte-Carlo: a number, "
                         "or 'auto' for the calibrated gate in result.json beside --params "
                         "(default 0.95 ln n)")
    ap.add_argument("--out", default="bbe_out/query_loop.json")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    params = np.load(args.params)
    gate = args.gate
    if gate == "auto":
        with open(os.path.join(os.path.dirname(args.params), "result.json")) as f:
            gate = json.load(f)["gate"]["entropy_threshold"]
    t0 = time.perf_counter()
    res = run(params, every=args.every, n_bettors=args.bettors, judge_sims=args.judge_sims,
              gate=None if gate is None else float(gate), max_rounds=args.max_rounds,
              log=lambda m: print(f"[query] {m}", flush=True))
    res["wall_s"] = time.perf_counter() - t0
    summary = {k: v for k, v in res.items() if k != "per_round"}
    print(json.dumps(summary), flush=True)
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
