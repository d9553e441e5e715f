"""Seeded synthetic inputs for the race workloads.

This module draws race descriptions, request sizes and in-play targets from
numpy's PCG64 generator.  It holds none of the race model's arithmetic: the
in-play states themselves are produced by running the model (on the GPU by
the library, on the CPU by the oracle), starting from the targets drawn here.
Both the GPU path and the CPU oracle take their inputs from here.

Recipe (the paper fixes no parameter ranges; it prints only the example step
laws U(10,20) and U(1,25), a 2000 m race lasting under six minutes, and
dt = 1 s for its timing runs -- Section 3 and the captions of Figs. 1 and 3):

* base speed mu ~ U(6.0, 7.5) distance units per second, so a 2000-unit race
  takes about 267-338 s;
* relative noise half-width sigma ~ U(1/3, 12/13): the paper's two examples
  have 5/15 and 12/13;
* step law delta = U(lo, hi) with lo = dt*mu*(1-sigma), hi = dt*mu*(1+sigma),
  computed in float64 and rounded to float32;
* responsiveness rho ~ U(-0.2, 0.2); preference coefficient 1; blocking
  threshold theta = 2 distance units.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TRACK_LEN = 2000.0
MAX_N = 20

# Named workloads (sizes and seeds).
CFG_START_N5 = dict(name="mc_start_n5_1e3", n=5, dt=1.0, param_seed=1, mc_seed=1, request=0,
                    n_sims=1000, stop_after=None)
CFG_START_N20 = dict(name="mc_start_n20_1e6", n=20, dt=1.0, param_seed=2, mc_seed=2, request=0,
                     n_sims=1_000_000, stop_after=None)
CFG_BATCH = dict(name="batch_inplay_4096", n_requests=4096, dt=1.0, seed=3, n_lo=5, n_hi=20,
                 frac_lo=0.05, frac_hi=1.0, sims_lo=100, sims_hi=10_000)
CFG_SURROGATE = dict(name="surrogate_train", dt=1.0, seed=4, n_lo=5, n_hi=20, p_n20=0.25,
                     frac_lo=0.05, frac_hi=1.0, label_sims=10_000)
CFG_QUERY = dict(name="inplay_query_loop", n=20, dt=1.0, seed=5, real_request=0xC0000000,
                 n_bettors=10_000, every=1, audit_frac=0.01, mc_sims=10_000, judge_sims=1_000_000)
CFG_VIEWS = dict(name="views_inplay_1e5", n_bettors=100_000, seed=6, ud_d_hi=30.0, linex_n_hi=60,
                 views_seed=7)

PREFIX_REQUEST_BIT = 0x80000000  # request ids used for the runs that produce in-play states


def competitor_params(rng: np.random.Generator, n: int, dt: float = 1.0) -> np.ndarray:
    """[n, 5] float32 rows (lo, hi, pref, rho, theta) per the recipe above."""
    mu = rng.uniform(6.0, 7.5, size=n)
    sigma = rng.uniform(1.0 / 3.0, 12.0 / 13.0, size=n)
    rho = rng.uniform(-0.2, 0.2, size=n)
    lo = dt * mu * (1.0 - sigma)
    hi = dt * mu * (1.0 + sigma)
    out = np.empty((n, 5), dtype=np.float32)
    out[:, 0] = lo
    out[:, 1] = hi
    out[:, 2] = 1.0
    out[:, 3] = rho
    out[:, 4] = 2.0
    return out


def pace_params(rng: np.random.Generator, comp: np.ndarray, gamma_hi: float = 0.0015,
                tau_hi: int = 300) -> np.ndarray:
    """Competitor rows with the time term of the responsiveness appended:
    [n, 7] float32, gamma ~ U(-gamma_hi, gamma_hi) per tick (fading or
    strengthening by up to 0.45 over a 300-tick race), tau ~ U{0..tau_hi}
    ticks."""
    n = comp.shape[0]
    out = np.zeros((n, 7), dtype=np.float32)
    out[:, :5] = comp
    out[:, 5] = rng.uniform(-gamma_hi, gamma_hi, size=n)
    out[:, 6] = rng.integers(0, tau_hi + 1, size=n)
    return out


def start_config(cfg: dict) -> dict:
    """A plain Monte-Carlo workload from the start line."""
    rng = np.random.default_rng(cfg["param_seed"])
    comp = competitor_params(rng, cfg["n"], cfg["dt"])
    stop = cfg["stop_after"] or cfg["n"]
    return dict(comp=comp, L=TRACK_LEN, n_sims=cfg["n_sims"], seed=cfg["mc_seed"],
                request=cfg["request"], stop_after=stop)


@dataclass
class RequestSpec:
    """One in-play request: race, where its state comes from, and its size."""
    index: int
    comp: np.ndarray          # [n, 5] float32
    remaining: float          # fraction of the track still ahead of the leader
    target: float             # leader position at which the in-play state is taken
    n_sims: int
    prefix_request: int       # request id of the run that produces the state
    prefix_sim: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.comp.shape[0])


def _log_uniform_int(rng, lo, hi) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_requests(cfg: dict = CFG_BATCH, n_requests: int | None = None) -> list[RequestSpec]:
    """Uneven in-play requests: n ~ U{n_lo..n_hi}, remaining ~ U(frac_lo, frac_hi)
    of the track for the leader, sims ~ log-uniform [sims_lo, sims_hi]."""
    n_requests = cfg["n_requests"] if n_requests is None else n_requests
    out = []
    for r in range(n_requests):
        rng = np.random.default_rng([cfg["seed"], r])
        n = int(rng.integers(cfg["n_lo"], cfg["n_hi"] + 1))
        comp = competitor_params(rng, n, cfg["dt"])
        rem = float(rng.uniform(cfg["frac_lo"], cfg["frac_hi"]))
        sims = _log_uniform_int(rng, cfg["sims_lo"], cfg["sims_hi"])
        target = np.float32(TRACK_LEN * (1.0 - rem))
        out.append(RequestSpec(index=r, comp=comp, remaining=rem, target=float(target),
                               n_sims=sims, prefix_request=PREFIX_REQUEST_BIT | r))
    return out


def cheap_bettors(cfg: dict = CFG_VIEWS, n_bettors: int | None = None):
    """Kinds (uint8: 0 ZI, 1 LW, 2 UD, 3 LinEx, a quarter each, shuffled)
    and parameters (float32) of a population of cheap in-play bettors: UD
    distance D uniform in [0, ud_d_hi] distance units (up to about four
    typical steps), LinEx window N a log-uniform integer in
    [1, linex_n_hi] ticks."""
    rng = np.random.default_rng(cfg["seed"])
    nb = int(n_bettors if n_bettors is not None else cfg["n_bettors"])
    kinds = (np.arange(nb) % 4).astype(np.uint8)
    rng.shuffle(kinds)
    params = np.zeros(nb, dtype=np.float32)
    ud = kinds == 2
    params[ud] = rng.uniform(0.0, cfg["ud_d_hi"], int(ud.sum()))
    lx = kinds == 3
    params[lx] = np.round(np.exp(rng.uniform(0.0, math.log(cfg["linex_n_hi"]), int(lx.sum()))))
    return kinds, params


def surrogate_states(n_states: int, cfg: dict = CFG_SURROGATE, first: int = 0) -> list[RequestSpec]:
    """Training / evaluation states for the surrogate: like the batched
    requests (dt = 1 s, the paper's timing step), with a quarter of the
    races at n = 20."""
    out = []
    for r in range(first, first + n_states):
        rng = np.random.default_rng([cfg["seed"], r])
        if rng.uniform() < cfg["p_n20"]:
            n = 20
        else:
            n = int(rng.integers(cfg["n_lo"], cfg["n_hi"] + 1))
        comp = competitor_params(rng, n, cfg["dt"])
        rem = float(rng.uniform(cfg["frac_lo"], cfg["frac_hi"]))
        target = np.float32(TRACK_LEN * (1.0 - rem))
        out.append(RequestSpec(index=r, comp=comp, remaining=rem, target=float(target),
                               n_sims=cfg["label_sims"],
                               prefix_request=PREFIX_REQUEST_BIT | (r & 0x7FFFFFFF)))
    return out


SURROGATE_BLOCK = 65536  # states per block of surrogate_state_block


def surrogate_state_block(block: int, count: int = SURROGATE_BLOCK,
                          cfg: dict = CFG_SURROGATE) -> dict:
    """Block `block` of the surrogate's states, drawn as arrays (the same
    recipe as surrogate_states, one generator per block, so that 10^7
    states take seconds): comp float32 [count, 20, 5] (zero rows past n),
    n int32 [count], target float32 [count] (leader position at which the
    state is taken), prefix_request uint32 [count] (request id of the run
    that produces the state: PREFIX_REQUEST_BIT | global state index)."""
    rng = np.random.default_rng([cfg["seed"], 0xB10C, block])
    n = np.where(rng.uniform(size=count) < cfg["p_n20"], 20,
                 rng.integers(cfg["n_lo"], cfg["n_hi"] + 1, size=count)).astype(np.int32)
    mu = rng.uniform(6.0, 7.5, size=(count, MAX_N))
    sigma = rng.uniform(1.0 / 3.0, 12.0 / 13.0, size=(count, MAX_N))
    rho = rng.uniform(-0.2, 0.2, size=(count, MAX_N))
    rem = rng.uniform(cfg["frac_lo"], cfg["frac_hi"], size=count)
    dt = cfg["dt"]
    comp = np.zeros((count, MAX_N, 5), dtype=np.float32)
    comp[:, :, 0] = dt * mu * (1.0 - sigma)
    comp[:, :, 1] = dt * mu * (1.0 + sigma)
    comp[:, :, 2] = 1.0
    comp[:, :, 3] = rho
    comp[:, :, 4] = 2.0
    comp[np.arange(MAX_N)[None, :] >= n[:, None]] = 0.0
    index = block * SURROGATE_BLOCK + np.arange(count, dtype=np.int64)
    return dict(comp=comp, n=n, target=(TRACK_LEN * (1.0 - rem)).astype(np.float32),
                prefix_request=(PREFIX_REQUEST_BIT | (index & 0x7FFFFFFF)).astype(np.uint32))


def query_race(cfg: dict = CFG_QUERY) -> dict:
    rng = np.random.default_rng(cfg["seed"])
    comp = competitor_params(rng, cfg["n"], cfg["dt"])
    return dict(comp=comp, L=TRACK_LEN, seed=cfg["seed"], real_request=cfg["real_request"])


SURROGATE_LAYERS = [(256, 160), (256, 256), (256, 256), (20, 256)]


def surrogate_random(seed: int) -> np.ndarray:
    """Surrogate parameters for checks: the weights of surrogate_init(seed)
    with non-zero biases, uniform in +-0.5 for the hidden layers and +-1 for
    the output layer."""
    p = surrogate_init(seed)
    rng = np.random.default_rng([seed, 0xB1A5])
    o = 0
    for i, (n, k) in enumerate(SURROGATE_LAYERS):
        o += n * k
        p[o:o + n] = rng.uniform(-1.0 if i == 3 else -0.5, 1.0 if i == 3 else 0.5, size=n)
        o += n
    return p


def surrogate_init(seed: int = 4) -> np.ndarray:
    """Initial surrogate parameters (packed W1, b1, ..., W4, b4, float32):
    weights uniform in +-sqrt(6/fan_in) (He-uniform for ReLU layers; the
    output layer uses +-sqrt(1/fan_in)), biases zero."""
    rng = np.random.default_rng([seed, 0x5EED])
    parts = []
    for i, (n, k) in enumerate(SURROGATE_LAYERS):
        bound = np.sqrt((1.0 if i == 3 else 6.0) / k)
        parts.append(rng.uniform(-bound, bound, size=n * k))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)
