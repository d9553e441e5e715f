#!/usr/bin/env python3
"""Throughput of the race Monte-Carlo on one MI355X.

Workload (one "step"): 10^6 simulations of a 20-competitor race on a
2000-unit track from the start line, full finish order resolved
(stop_after = 20), tallied into win counts and win probabilities -- the
whole hot path (bbe_race_sim + bbe_win_probs) over one batch.  Inputs are
seeded and synthetic (paper_2108_02419_amd/inputs.py); every step uses a
new Monte-Carlo seed.

Prints ONE JSON line.  `value` is simulations per second; the roofline
object prices the Monte-Carlo kernel against the vector-ALU issue peak of
the chip (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: a wave64 vector
instruction occupies its SIMD for four cycles) using the algorithmic
instruction count per competitor-step, and takes the HBM traffic per launch
from the committed counter profile when that profile was taken on the
current kernel sources; the cpu_baseline object times the
CPU oracle on a bounded sample of the same workload (cpu_baselines_other:
the other workloads, on bounded samples).  `winner_only` times the same
workload resolved only to each simulation's winner (the same win counts).
More objects measure the other
workloads of the path: `cfg0` (5 competitors, 10^3 simulations), `batch`
(4096 uneven in-play requests in one graph-captured persistent launch),
`surrogate` (queries per second of the surrogate network against
Monte-Carlo at 10^4 simulations per query, on the same in-play state),
`bettors` (10^4 RP(d) bettors re-running their dry-runs every tick of an
in-play race) and `surrogate_gated` (the trained network, gated to the 0.02
error target by the pooled 1% audit, over a whole in-play query loop; the
same for races of 0.1-second ticks queried every 10 ticks in
`surrogate_gated_dt01`).
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

# Algorithmic vector work per competitor-step, in wave64 vector-instruction
# issue slots (each 32x32->64 product is one v_mad_u64_u32, each three-way
# xor one v_bitop3_b32): an eighth of one Philox4x32-10 block (20 products
# and 20 xors serve the block's 8 draws: 2.5 + 2.5), the draw's conversion
# (1), Eq. 1 (R 2, free step 2, min 1, product 1, gap 1, test 1, select 1 =
# 9), the update and finish test (3), and the competitor-ahead query with a
# maintained order (carry past equal positions 3, one order check 1).
ALGO_OPS_PER_COMPETITOR_STEP = 22.0
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9  # lane-instr/s: CUs x SIMDs x lanes/clock x clock

# The counter profile of the Monte-Carlo kernel on this workload, and the
# sources it was taken on.
PROFILE = os.path.join(ROOT, "profiles", "race_mc_kernel_n20_1e6.md")
KERNEL_SOURCES = ["race_kernels.hip", "race_mc.hpp", "race_sim.hpp", "race_common.hpp",
                  "kernels.hpp"]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_02419_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_values() -> dict:
    """Figures of the committed profile of the dominant kernel, keyed by
    their header names (kernel_sources_sha256, traffic_bytes_per_launch,
    valu_busy_pct, ...), or {} if the profile is missing or was taken on
    other kernel sources."""
    try:
        with open(PROFILE) as f:
            text = f.read()
    except OSError:
        return {}
    vals = {}
    for line in text.splitlines():
        line = line.strip().strip("`")
        key, sep, val = line.partition(":")
        if sep and key and " " not in key and key == key.lower() and val.strip():
            vals.setdefault(key, val.strip())
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256():
        return {}
    return vals


def profiled_float(name: str):
    try:
        return float(profiled_values()[name])
    except (KeyError, ValueError):
        return None


def profiled_traffic():
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the copy-probe
    factors) from the committed profile, or None if the profile is missing or
    was taken on other kernel sources."""
    return profiled_float("traffic_bytes_per_launch")


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
    sample = int(min(max(probe, probe * target_s / max(dt, 1e-6)), 800_000))
    t0 = time.perf_counter()
    _, wins, steps = oracle.race_sim(c["comp"], c["L"], sample, c["seed"], request=c["request"],
                                     stop_after=c["stop_after"], want_orders=False,
                                     threads=threads)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, on a fortieth of that sample
    one = max(200, sample // 40)
    t1 = time.perf_counter()
    _, _, steps1 = oracle.race_sim(c["comp"], c["L"], one, c["seed"], request=c["request"],
                                   stop_after=c["stop_after"], want_orders=False, threads=1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"value": sample / dt, "unit": "sims/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} simulations of the same workload "
                      f"({steps} competitor-steps, {dt:.2f} s)",
            "competitor_steps_per_s": steps / dt,
            "single_thread": {"value": one / dt1, "unit": "sims/s",
                              "sample": f"first {one} simulations ({dt1:.2f} s)",
                              "competitor_steps_per_s": steps1 / dt1},
            "host": {"cpu_model": model, "nproc": os.cpu_count()}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-gated", action="store_true",
                    help="skip the trained, gated surrogate leg")
    ap.add_argument("--no-bettors", action="store_true",
                    help="skip the RP(d) bettor-population leg")
    ap.add_argument("--stop-after", type=int, default=None,
                    help="finishers to resolve per simulation (default: all 20)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one plain device-to-device copy of this many MiB "
                         "(a reference for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the Monte-Carlo "
              "shards by simulation range across GPUs, but bench.py measures a single GPU.",
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
    # the same launch with the finish-order matrix written ([n_sims][n] uint8)
    orders = torch.empty((n_sims, n), dtype=torch.uint8, device=dev)
    oev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(8)]
    for k, (ea, eb) in enumerate(oev):  # the first launch touches the matrix first: not timed
        ea.record(stream)
        _bbe.race_sim(race, n_sims, c["seed"] + k, request=c["request"],
                      stop_after=c["stop_after"], orders=orders, wins=wins,
                      steps=steps_t[0], stream=stream)
        eb.record(stream)
    torch.cuda.synchronize()
    orders_ms = sorted(a.elapsed_time(b) for a, b in oev[1:])[3]
    # finish-position tallies of that matrix (place probabilities)
    counts = torch.empty((n, n), dtype=torch.int64, device=dev)
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _bbe.rank_counts(orders, n, counts, stream=stream)
    ea.record(stream)
    _bbe.rank_counts(orders, n, counts, stream=stream)
    eb.record(stream)
    torch.cuda.synchronize()
    rank_counts_ms = ea.elapsed_time(eb)
    assert int(counts.sum().item()) == n_sims * n
    del orders

    # the same workload resolved only to its winner (stop_after = 1): the
    # win counts and probabilities are the same as with the full order
    wev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(8)]
    w_steps = []
    _bbe.race_sim(race, n_sims, c["seed"], request=c["request"], stop_after=c["stop_after"],
                  wins=wins, steps=steps_t[0], stream=stream)
    torch.cuda.synchronize()
    wins_full = wins.clone()
    for k, (ea, eb) in enumerate(wev):
        ea.record(stream)
        _bbe.race_sim(race, n_sims, c["seed"], request=c["request"], stop_after=1,
                      wins=wins, steps=steps_t[0], stream=stream)
        eb.record(stream)
        torch.cuda.synchronize()
        w_steps.append(int(steps_t[0].item()))
    assert torch.equal(wins, wins_full)  # the same winners as the full order
    w_ms = sorted(a.elapsed_time(b) for a, b in wev[1:])
    w_med = w_ms[len(w_ms) // 2]
    winner_only = {"workload": "mc_start_n20_1e6 resolved to the winner only (stop_after 1)",
                   "kernel_ms": w_med, "sims_per_s": n_sims / (w_med / 1e3),
                   "competitor_steps_per_launch": w_steps[-1],
                   "competitor_steps_per_s": w_steps[-1] / (w_med / 1e3),
                   "frac": w_steps[-1] * ALGO_OPS_PER_COMPETITOR_STEP / (w_med / 1e3)
                   / VALU_PEAK_OPS}

    # the same workload with a time term in every competitor's responsiveness
    # (the paced kernel variant): kernel time and competitor-steps per second
    import numpy as np
    paced_comp = inputs.pace_params(np.random.default_rng(2), c["comp"])
    paced_race = Race(paced_comp, c["L"])
    pev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(4)]
    p_steps = []
    for k, (ea, eb) in enumerate(pev):
        ea.record(stream)
        _bbe.race_sim(paced_race, n_sims, c["seed"] + k, request=c["request"],
                      stop_after=c["stop_after"], wins=wins, steps=steps_t[0], stream=stream)
        eb.record(stream)
        torch.cuda.synchronize()
        p_steps.append(int(steps_t[0].item()))
    p_ms = [a.elapsed_time(b) for a, b in pev[1:]]
    paced = {"workload": "mc_start_n20_1e6 with gamma ~ U(-0.0015, 0.0015), tau ~ U{0..300}",
             "kernel_ms": sorted(p_ms)[1],
             "competitor_steps_per_s": sum(p_steps[1:]) / (sum(p_ms) / 1e3)}

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
        "with_orders_kernel_ms": orders_ms,
        "rank_counts_ms": rank_counts_ms,
        "winner_only": winner_only,
        "paced": paced,
        "wall_s": wall,
        "device": {"name": torch.cuda.get_device_name(0),
                   "cus": torch.cuda.get_device_properties(0).multi_processor_count},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": profiled_traffic(),
                     "instr_per_competitor_step": ALGO_OPS_PER_COMPETITOR_STEP,
                     # rocprofv3 counters of the same kernel sources (null if stale)
                     "valu_busy_pct": profiled_float("valu_busy_pct"),
                     "valu_lane_activity_pct": profiled_float("valu_lane_activity_pct")},
    }
    line["cfg0"] = cfg0_leg()
    if not args.no_batch:
        line["batch"] = batch_leg(args.batch_steps)
    if not args.no_surrogate:
        line["surrogate"] = surrogate_leg()
    if not args.no_bettors:
        line["bettors"] = bettors_leg()
        line["views"] = views_leg()
    if not args.no_gated:
        line["surrogate_gated"] = gated_leg()
        # the query loop as first specified: 0.1-second ticks, a round every
        # 10 ticks (the plain path timed on every 30th round)
        line["surrogate_gated_dt01"] = gated_leg(trained=TRAINED_DT01, dt=0.1, every=10,
                                                 baseline_every=30)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c)
        line["cpu_baselines_other"] = cpu_baselines(line["cpu_baseline"]["cores"])
    print(json.dumps(line), flush=True)
    return 0


def cfg0_leg(reps: int = 20):
    """The small start workload (5 competitors, 10^3 simulations, finish
    orders and win counts): median kernel time of `reps` launches."""
    import numpy as np
    import torch

    from paper_2108_02419_amd import _bbe, inputs
    c = inputs.start_config(inputs.CFG_START_N5)
    race = _bbe.Race(c["comp"], c["L"])
    dev = torch.device("cuda", 0)
    orders = torch.empty((c["n_sims"], race.n), dtype=torch.uint8, device=dev)
    wins = torch.empty(race.n, dtype=torch.int64, device=dev)
    st = torch.empty(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def launch():
        _bbe.race_sim(race, c["n_sims"], c["seed"], request=c["request"], orders=orders,
                      wins=wins, steps=st, stream=stream)

    for _ in range(3):
        launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        launch()
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)
    med = ms[len(ms) // 2] / 1e3
    csteps = int(st.item())
    assert int(wins.sum().item()) == c["n_sims"]
    return {"workload": "mc_start_n5_1e3: 5 competitors, track 2000, 10^3 sims from the start, "
                        "finish orders + win counts",
            "kernel_ms": {"median": med * 1e3, "min": ms[0],
                          "cov": float(np.std(ms) / np.mean(ms))},
            "sims_per_s": c["n_sims"] / med, "competitor_steps": csteps,
            "competitor_steps_per_s": csteps / med,
            "note": "one generation of 64 simulations per wave: 16 waves on a 1024-wave chip, "
                    "so the launch is latency-bound"}


def cpu_baselines(threads: int):
    """The oracle on bounded samples of the other workloads (states from the
    oracle's own runs), each with what it extrapolates to."""
    import numpy as np

    import oracle
    from paper_2108_02419_amd import inputs
    out = {}
    L = inputs.TRACK_LEN
    c0 = inputs.start_config(inputs.CFG_START_N5)
    t0 = time.perf_counter()
    _, _, st = oracle.race_sim(c0["comp"], L, c0["n_sims"], c0["seed"], request=c0["request"],
                               threads=threads)
    dt = time.perf_counter() - t0
    out["mc_start_n5_1e3"] = {"value": c0["n_sims"] / dt, "unit": "sims/s", "cores": threads,
                              "kind": "oracle", "sample": "the whole workload (1000 sims)",
                              "competitor_steps_per_s": st / dt}
    # uneven batch: the first 192 of the 4096 requests, in full
    reqs = inputs.batch_requests(n_requests=192)
    states = [oracle.race_prefix(r.comp, L, inputs.CFG_BATCH["seed"], r.prefix_request, 0,
                                 r.target) for r in reqs]
    t0 = time.perf_counter()
    sims = steps = 0
    for r, s in zip(reqs, states):
        _, _, st = oracle.race_sim(r.comp, L, r.n_sims, inputs.CFG_BATCH["seed"],
                                   request=r.index, state=s, want_orders=False, threads=threads)
        sims += r.n_sims
        steps += st
    dt = time.perf_counter() - t0
    full = sum(r.n_sims for r in inputs.batch_requests())
    out["batch_inplay_4096"] = {
        "value": sims / dt, "unit": "sims/s", "cores": threads, "kind": "oracle",
        "sample": f"first 192 of 4096 requests in full ({sims} sims, {steps} competitor-steps, "
                  f"{dt:.2f} s)", "competitor_steps_per_s": steps / dt,
        "extrapolated_full_s": dt * full / sims}
    # surrogate labels: 64 training states x 10^4 sims, winner only
    a = inputs.surrogate_state_block(0, 64)
    t0 = time.perf_counter()
    steps = 0
    for i in range(64):
        comp = a["comp"][i, :a["n"][i]]
        s = oracle.race_prefix(comp, L, inputs.CFG_SURROGATE["seed"], int(a["prefix_request"][i]),
                               0, float(a["target"][i]))
        _, _, st = oracle.race_sim(comp, L, 10_000, inputs.CFG_SURROGATE["seed"], request=i,
                                   state=s, stop_after=1, want_orders=False, threads=threads)
        steps += st
    dt = time.perf_counter() - t0
    out["surrogate_labels"] = {
        "value": 64 / dt, "unit": "labelled states/s", "cores": threads, "kind": "oracle",
        "sample": f"64 training states x 10^4 sims, winner only ({steps} competitor-steps, "
                  f"{dt:.2f} s)", "competitor_steps_per_s": steps / dt,
        "extrapolated_1e7_states_h": dt / 64 * 1e7 / 3600}
    # in-play Monte-Carlo queries: 10 queries x 10^4 sims on the query race at tick 100
    q = inputs.query_race()
    trace = oracle.race_trace(q["comp"], L, q["seed"], q["real_request"], 0, 101)
    s = oracle.race_prefix(q["comp"], L, q["seed"], q["real_request"], 0,
                           np.float32(trace[100].max()))
    t0 = time.perf_counter()
    steps = 0
    for i in range(10):
        _, _, st = oracle.race_sim(q["comp"], L, 10_000, q["seed"] + 1, request=i, state=s,
                                   stop_after=1, want_orders=False, threads=threads)
        steps += st
    dt = time.perf_counter() - t0
    out["query_mc"] = {"value": 10 / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
                       "sample": f"10 queries x 10^4 sims at tick {s[0]} of the query race "
                                 f"({steps} competitor-steps, {dt:.2f} s)",
                       "competitor_steps_per_s": steps / dt}
    return out


def batch_leg(steps: int):
    """4096 uneven in-play requests (states from the GPU generator), one
    autotuned plan, `steps` timed graph launches."""
    import numpy as np
    import torch

    from paper_2108_02419_amd import _bbe, inputs
    reqs = inputs.batch_requests()
    races = [_bbe.Race(r.comp, inputs.TRACK_LEN) for r in reqs]
    n = len(reqs)
    dev = torch.device("cuda", 0)
    tick = torch.empty(n, dtype=torch.int32, device=dev)
    pos = torch.empty((n, 20), dtype=torch.float32, device=dev)
    prev = torch.empty((n, 20), dtype=torch.float32, device=dev)
    seed = inputs.CFG_BATCH["seed"]
    _bbe.prefix_batch([(race, None, 0, 1, r.prefix_request, 0) for r, race in zip(reqs, races)],
                      np.zeros(n, np.uint32), [r.target for r in reqs], seed, tick, pos, prev)
    T, P, V = tick.cpu().numpy().view(np.uint32), pos.cpu().numpy(), prev.cpu().numpy()
    specs = [(race, (int(T[i]), P[i, :r.n].copy(), V[i, :r.n].copy()), 0, r.n_sims, r.index, 0)
             for i, (r, race) in enumerate(zip(reqs, races))]
    wins = torch.zeros((n, 20), dtype=torch.int64, device=dev)
    probs = torch.zeros((n, 20), dtype=torch.float64, device=dev)
    stc = torch.zeros(1, dtype=torch.int64, device=dev)
    t0 = time.perf_counter()
    plan = _bbe.BatchPlan(specs, seed, wins, probs, stc, autotune=True)
    setup_s = time.perf_counter() - t0
    plan.launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record()
        plan.launch()
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)
    sims = sum(r.n_sims for r in reqs)
    csteps = int(stc.item())
    med = ms[len(ms) // 2] / 1e3
    assert int(wins.sum().item()) == sims
    return {"workload": "batch_inplay_4096: 4096 requests, n 5-20, remaining 5-100% of 2000, "
                        "100-10^4 sims each, full finish order, one persistent graph launch",
            "requests": n, "sims": sims, "competitor_steps": csteps,
            "ms_per_launch": {"median": ms[len(ms) // 2], "min": ms[0],
                              "cov": float(np.std(ms) / np.mean(ms))},
            "sims_per_s": sims / med, "competitor_steps_per_s": csteps / med,
            "alu_frac": csteps * ALGO_OPS_PER_COMPETITOR_STEP / med / VALU_PEAK_OPS,
            "plan": plan.info(), "plan_setup_s": setup_s}


def surrogate_leg(n_queries: int = 10_000, mc_queries: int = 10_000, mc_sims: int = 10_000):
    """Queries per second: the surrogate (encode + forward on 10^4 queries)
    against Monte-Carlo (the same 10^4 queries as distinct requests of one
    batched plan, 10^4 simulations each, winner only), on one
    in-play state of the 20-competitor query race (dt = 1 s, 100 ticks
    in, about a third of the race).  The network has its seeded initial weights: throughput does not
    depend on training."""
    import numpy as np
    import torch

    from paper_2108_02419_amd import _bbe, inputs
    q = inputs.query_race()
    comp, n = q["comp"], q["comp"].shape[0]
    race = _bbe.Race(comp, inputs.TRACK_LEN)
    dev = torch.device("cuda", 0)
    tick = torch.empty(1, dtype=torch.int32, device=dev)
    pos = torch.empty(n, dtype=torch.float32, device=dev)
    prev = torch.empty(n, dtype=torch.float32, device=dev)
    _bbe.race_advance(race, q["seed"], q["real_request"], 0, 100, tick, pos, prev)
    torch.cuda.synchronize()
    state = (int(tick.item()), pos.cpu().numpy(), prev.cpu().numpy())
    net = _bbe.Mlp(inputs.surrogate_init(), max_batch=8)
    comp_b = torch.tensor(np.broadcast_to(np.pad(comp, ((0, 20 - n), (0, 0))),
                                          (n_queries, 20, 5)).copy(), device=dev)
    n_b = torch.full((n_queries,), n, dtype=torch.int32, device=dev)
    pos_b = torch.zeros((n_queries, 20), dtype=torch.float32, device=dev)
    prev_b = torch.zeros((n_queries, 20), dtype=torch.float32, device=dev)
    pos_b[:, :n] = pos
    prev_b[:, :n] = prev
    x = torch.empty((n_queries, 160), dtype=torch.int16, device=dev)
    sp = torch.empty((n_queries, 20), dtype=torch.float32, device=dev)
    se = torch.empty(n_queries, dtype=torch.float32, device=dev)

    def sur():
        _bbe.encode_states(comp_b, n_b, pos_b, prev_b, inputs.TRACK_LEN,
                           inputs.CFG_QUERY["dt"], x)
        net.forward(x, n_b, sp, se)

    for _ in range(3):
        sur()
    torch.cuda.synchronize()
    reps = 20
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        sur()
    b.record()
    torch.cuda.synchronize()
    sur_s = a.elapsed_time(b) / 1e3 / reps
    specs = [(race, state, 0, mc_sims, i, 1) for i in range(mc_queries)]
    wins = torch.zeros((mc_queries, 20), dtype=torch.int64, device=dev)
    probs = torch.zeros((mc_queries, 20), dtype=torch.float64, device=dev)
    plan = _bbe.BatchPlan(specs, q["seed"] + 1, wins, probs, None, autotune=True)
    plan.launch()
    torch.cuda.synchronize()
    a.record()
    for _ in range(3):
        plan.launch()
    b.record()
    torch.cuda.synchronize()
    mc_s = a.elapsed_time(b) / 1e3 / 3
    sq, mq = n_queries / sur_s, mc_queries / mc_s
    return {"workload": f"query race n=20, dt 1 s, state at tick 100; surrogate: {n_queries} "
                        f"queries (encode + forward); MC: {mc_queries} queries x {mc_sims} sims "
                        f"(one batched plan), winner only",
            "surrogate_queries_per_s": sq, "mc_queries_per_s": mq, "speedup": sq / mq,
            "surrogate_ms_per_launch": sur_s * 1e3, "mc_ms_per_launch": mc_s * 1e3}


def bettors_leg(n_bettors: int = 10_000, d_lo: int = 1, d_hi: int = 200, n_cheap: int = 100_000):
    """RP(d) bettors updating once per tick through a whole in-play race:
    10^4 bettors, d log-uniform in [1, 200], one plan re-pointed at each new
    state; GPU time of the plan launches.  Beside them 10^5 cheap bettors
    (LinEx, LW, UD, ZI) re-form their views every tick from the race's
    trace, and the RP(d) bettors' views are read off their win counts."""
    from paper_2108_02419_amd import bettors
    r = bettors.run(n_bettors, d_lo, d_hi, n_cheap=n_cheap)
    return {"workload": f"{n_bettors} RP(d) bettors, d log-uniform in [{d_lo}, {d_hi}] "
                        f"(mean {r['d_mean']:.1f}), every tick of the n=20 query race "
                        f"({r['rounds']} rounds); {n_cheap} LinEx/LW/UD/ZI bettors",
            "dry_runs_per_s": r["dry_runs_per_s"], "bettor_updates_per_s": r["bettor_updates_per_s"],
            "gpu_ms_per_round": r["gpu_ms_per_round"], "dry_runs": r["dry_runs"],
            "host_ms_per_round_set_states": 1e3 * r["host_seconds_set_states"] / max(1, r["rounds"]),
            "views_gpu_ms_per_round": r["views_gpu_ms_per_round"],
            "backing_winner_by_tick": r["backing_winner_by_tick"],
            "plan": r["plan"]}


def views_leg(steps: int = 20):
    """Views of 10^5 cheap bettors (a quarter each LinEx, LW, UD, ZI) at
    every tick of the n=20 query race's trace, in one launch; plus the views
    of 10^4 RP(d) bettors from their win counts."""
    import numpy as np
    import torch

    from paper_2108_02419_amd import _bbe, api, inputs
    q = inputs.query_race()
    race = _bbe.Race(q["comp"], inputs.TRACK_LEN)
    trace = api.trace(race, q["seed"], q["real_request"], 0, 1 << 16)
    rows, n = trace.shape
    kinds, params = inputs.cheap_bettors()
    nb = int(kinds.size)
    b = _bbe.Bettors(kinds, params)
    dev = trace.device
    views = torch.empty((rows, nb), dtype=torch.uint8, device=dev)
    counts = torch.empty((rows, n), dtype=torch.int32, device=dev)
    seed = inputs.CFG_VIEWS["views_seed"]

    def launch():
        b.views(trace, rows, inputs.TRACK_LEN, 0, seed, 0, rows, views=views, counts=counts)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for e0, e1 in evs:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))

    ms = timed(launch)
    n_rp = 10_000
    rng = np.random.default_rng(2)
    wins = torch.tensor(rng.integers(0, 50, (n_rp, 20)), dtype=torch.int64, device=dev)
    rp_v = torch.empty(n_rp, dtype=torch.uint8, device=dev)
    rp_c = torch.empty(n, dtype=torch.int32, device=dev)
    rp_ms = timed(lambda: _bbe.rp_views(wins, n, views=rp_v, counts=rp_c))
    n_views = rows * nb
    out_bytes = n_views + rows * n * 4
    return {"workload": f"views_inplay_1e5: {nb} cheap bettors (LinEx N 1-60, UD D 0-30, LW, ZI; "
                        f"a quarter each) x {rows} ticks of the n=20 query race, one launch",
            "ms_per_launch": ms, "views_per_s": n_views / (ms / 1e3),
            "output_gb_per_s": out_bytes / (ms / 1e3) / 1e9,
            "per_kind": [int(x) for x in b.per_kind()],
            "rp_views_10k_ms": rp_ms}


TRAINED = os.path.join(ROOT, "paper_2108_02419_amd", "trained", "surrogate.bbemlp")
TRAINED_DT01 = os.path.join(ROOT, "paper_2108_02419_amd", "trained", "surrogate_dt01.bbemlp")


def gated_leg(eval_states: int = 1000, judge_sims: int = 1_000_000, audit_tol: float = 0.0175,
              trained: str = TRAINED, dt: float = 1.0, every: int = 1, baseline_every: int = 10):
    """Surrogate vs Monte-Carlo queries per second at the error target, with
    the network trained by paper_2108_02419_amd.surrogate (its file and
    recipe in paper_2108_02419_amd/trained/): first judged afresh on held-out
    in-play states (max abs error against 10^6-simulation Monte-Carlo), then
    run through the whole in-play query loop: 10^4 bettors every round; the
    surrogate serves a round when its entropy is below 0.95 ln n and it
    agrees with the pooled 1% audit (10^4 simulations per audited bettor)
    within audit_tol, else every bettor gets its own Monte-Carlo answer --
    at the strict size that keeps every answer within 0.02 of the truth
    (query_loop.strict_sims; the headline figures), and, timed on the same
    rounds, at the plain path's 10^4 simulations (`fallback_1e4`); the plain
    Monte-Carlo path (every bettor at 10^4 simulations) is timed on every
    `baseline_every`-th round.  `dt` (seconds per tick) and `every` (ticks
    per round) select the race's time step; `trained` is the network trained
    at that step."""
    import torch

    from paper_2108_02419_amd import _bbe, inputs, query_loop, surrogate
    if not os.path.exists(trained):
        return {"skipped": f"{trained} missing"}
    net = _bbe.Mlp.load(trained, max_batch=8)
    t0 = time.perf_counter()
    # held-out states from blocks the training never used
    ex, en, jt, ans = surrogate.build_eval_set(eval_states, judge_sims, 4,
                                               fallback_sims=(10_000,),
                                               block0=surrogate.EVAL_BLOCK0 + 64,
                                               cfg=dict(inputs.CFG_SURROGATE, dt=dt))
    pred, ent = surrogate.predict(net, ex, en)
    torch.cuda.synchronize()
    heldout = {"states": eval_states, "judge_sims": judge_sims,
               "surrogate": surrogate.errors(pred, jt, en),
               "mc_1e4": surrogate.errors(ans[10_000], jt, en)}
    judge_s = time.perf_counter() - t0
    t1 = time.perf_counter()
    loop = query_loop.run(net, every=every, judge_sims=judge_sims,
                          fallback_sims=[10_000, "strict"], audit_tol=audit_tol,
                          baseline_every=baseline_every,
                          log=lambda m: print(f"[query] {m}", flush=True),
                          cfg=dict(inputs.CFG_QUERY, dt=dt))
    loop_s = time.perf_counter() - t1
    plain, strict = loop["fallbacks"]
    # the headline figures are those of the strict fallback: the system
    # whose every answer is held to the 0.02 target; the 10^4-simulation
    # fallback (the Monte-Carlo path's own answers) is reported beside it
    return {"workload": f"query race n=20, dt {dt} s, {loop['rounds']} rounds (every {every} "
                        f"ticks) x {loop['bettors']} bettors; "
                        f"surrogate from {os.path.relpath(trained, ROOT)}; audit 1% at "
                        f"{loop['mc_sims']} sims, pooled, tolerance {audit_tol}; fallback "
                        f"per bettor at the strict size (every answer within 0.02) and, on the "
                        f"same rounds, at 10^4 sims; judge {judge_sims} sims",
            "system_queries_per_s": strict["system_queries_per_s"],
            "mc_queries_per_s": loop["mc_queries_per_s"],
            "system_speedup": strict["system_speedup"],
            "answer_err_max": strict["answer_err"]["max"],
            "answer_err": strict["answer_err"],
            "fallback_mean_sims": strict["mean_sims"],
            "fallback_err": strict["fallback_err"],
            "fallback_1e4": {"note": "the same rounds with every flagged bettor answered at "
                                     "10^4 simulations, the Monte-Carlo path's own answers "
                                     "(their noise exceeds 0.02 on some states)",
                             "system_queries_per_s": plain["system_queries_per_s"],
                             "system_speedup": plain["system_speedup"],
                             "answer_err_max": plain["answer_err"]["max"],
                             "answer_err": plain["answer_err"],
                             "fallback_err": plain["fallback_err"]},
            "served_frac": loop["served_frac"],
            "served_err": loop["served_err"],
            "audit_mc_err": loop["mc_err"],
            "surrogate_raw_speedup": loop["speedup"],
            "surrogate_raw_err": loop["surrogate_err"],
            "seconds": loop["seconds"],
            "heldout": heldout,
            "heldout_judge_s": judge_s, "loop_s": loop_s}


if __name__ == "__main__":
    sys.exit(main())
