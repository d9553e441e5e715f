#!/usr/bin/env python3
"""Throughput of the race Monte-Carlo on one MI355X.

Workload (one "step"): 10^6 simulations of a 20-competitor race on a
2000-unit track from the start line, full finish order resolved
(stop_after = 20), tallied into win counts and win probabilities -- the
whole hot path (bbe_race_sim + bbe_win_probs) over one batch.  Inputs are
seeded and synthetic (paper_2108_02419_amd/inputs.py); every step uses a
new Monte-Carlo seed.

Prints ONE JSON line.  `value` is simulations per second; the roofline
object prices the Monte-Carlo kernel against the VALU peak of the chip
(256 CUs x 64 lanes x 2.4 GHz, full-rate lane operations) using the
algorithmic cost per competitor-step; the cpu_baseline object times the
CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU work per competitor-step, in full-rate lane-operation
# equivalents: a quarter of one Philox4x32-10 block (the draw), the
# competitor-ahead query with a maintained order, Eq. 1 and the update.
ALGO_OPS_PER_COMPETITOR_STEP = 48.0
VALU_PEAK_OPS = 256 * 64 * 2.4e9  # lane-ops/s: CUs x lanes x clock


def cpu_baseline(c, target_s: float = 12.0):
    import numpy as np  # noqa: F401

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    probe = 2000
    t0 = time.perf_counter()
    oracle.race_sim(c["comp"], c["L"], probe, c["seed"], request=c["request"],
                    stop_after=c["stop_after"], want_orders=False, threads=threads)
    dt = time.perf_counter() - t0
    sample = int(min(max(probe, probe * target_s / max(dt, 1e-6)), 200_000))
    t0 = time.perf_counter()
    _, wins, steps = oracle.race_sim(c["comp"], c["L"], sample, c["seed"], request=c["request"],
                                     stop_after=c["stop_after"], want_orders=False,
                                     threads=threads)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "sims/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} simulations of the same workload "
                      f"({steps} competitor-steps, {dt:.2f} s)",
            "competitor_steps_per_s": steps / dt}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stop-after", type=int, default=None,
                    help="finishers to resolve per simulation (default: all 20)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one plain device-to-device copy of this many MiB "
                         "(a reference for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the Monte-Carlo "
              "shards by simulation range across GPUs but this build measures a single GPU.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2108_02419_amd import api, inputs
    from paper_2108_02419_amd._bbe import Race

    torch.cuda.set_device(0)
    c = inputs.start_config(inputs.CFG_START_N20)
    if args.stop_after:
        c["stop_after"] = args.stop_after
    race = Race(c["comp"], c["L"])
    n_sims, n = c["n_sims"], race.n

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup
    wins = torch.empty(n, dtype=torch.int64, device=dev)
    steps_t = [torch.empty(1, dtype=torch.int64, device=dev) for _ in range(max(K, 1))]
    probs = torch.empty(n, dtype=torch.float64, device=dev)

    from paper_2108_02419_amd import _bbe

    def one_step(k, seed, ev=None):
        if ev is not None:
            ev[0].record(stream)
        _bbe.race_sim(race, n_sims, seed, request=c["request"], stop_after=c["stop_after"],
                      wins=wins, steps=steps_t[k % len(steps_t)], stream=stream)
        if ev is not None:
            ev[1].record(stream)
        _bbe.win_probs(wins, probs, stream=stream)

    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for w in range(W):
        one_step(0, 10_000 + w)
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(K):
        one_step(k, c["seed"] + k, evs[k])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    comp_steps = [int(t.item()) for t in steps_t[:K]]
    assert int(wins.sum().item()) == n_sims

    secs = total_ms / 1e3
    sims_per_s = K * n_sims / secs
    csteps_per_s = sum(comp_steps) / secs
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    avg_csteps = sum(comp_steps) / len(comp_steps)
    achieved = avg_csteps * ALGO_OPS_PER_COMPETITOR_STEP / avg_kern_s
    km = sorted(kern_ms)
    mean = sum(km) / len(km)
    cov = (sum((x - mean) ** 2 for x in km) / len(km)) ** 0.5 / mean if len(km) > 1 else 0.0

    line = {
        "metric": "race sims/s and competitor-steps/s (% VALU peak)",
        "value": sims_per_s,
        "unit": "sims/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": total_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mc_start_n20_1e6: 20 competitors, track 2000, 10^6 sims from "
                               "the start, win counts + probabilities",
                   "n_competitors": n, "n_sims": n_sims, "track_len": c["L"],
                   "stop_after": c["stop_after"], "param_seed": 2, "mc_seed": c["seed"]},
        "competitor_steps_per_s": csteps_per_s,
        "competitor_steps_per_step": avg_csteps,
        "kernel_ms": {"median": km[len(km) // 2], "mean": mean, "min": km[0], "cov": cov},
        "wall_s": wall,
        "device": {"name": torch.cuda.get_device_name(0),
                   "cus": torch.cuda.get_device_properties(0).multi_processor_count},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "ops_per_competitor_step": ALGO_OPS_PER_COMPETITOR_STEP},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
