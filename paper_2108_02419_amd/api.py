"""Tensor-level helpers over the C ABI: allocate the output tensors on the
current CUDA device and enqueue the library calls on the current stream.

Every computation runs in the library's kernels; these helpers only size
buffers and marshal arguments.
"""
from __future__ import annotations

import torch

from . import _bbe
from ._bbe import Race


def mc(race: Race, n_sims: int, seed: int, request: int = 0, state=None, sim_begin: int = 0,
       stop_after: int | None = None, want_orders: bool = False, want_steps: bool = True,
       stream=None, device=None):
    """Monte-Carlo dry-runs of one race.  Returns a dict of CUDA tensors:
    ``wins`` (int64 [n]), ``steps`` (int64 [1] or None), ``orders`` (uint8
    [n_sims, n] or None)."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    wins = torch.empty(race.n, dtype=torch.int64, device=dev)
    steps = torch.empty(1, dtype=torch.int64, device=dev) if want_steps else None
    orders = (torch.empty((n_sims, race.n), dtype=torch.uint8, device=dev)
              if want_orders else None)
    _bbe.race_sim(race, n_sims, seed, request=request, state=state, sim_begin=sim_begin,
                  stop_after=stop_after, orders=orders, wins=wins, steps=steps, stream=stream)
    return dict(wins=wins, steps=steps, orders=orders)


def win_probs(wins: torch.Tensor, n: int | None = None, stream=None) -> torch.Tensor:
    probs = torch.empty(wins.shape, dtype=torch.float64, device=wins.device)
    _bbe.win_probs(wins, probs, n=n, stream=stream)
    return probs


def prefix(race: Race, seed: int, request: int, sim: int, target: float, state=None,
           stream=None, device=None):
    """In-play state after advancing one simulation until the leader reaches
    ``target``.  Returns CUDA tensors (tick uint32-in-int32 [1], pos [n],
    prev [n])."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    tick = torch.empty(1, dtype=torch.int32, device=dev)
    pos = torch.empty(race.n, dtype=torch.float32, device=dev)
    prev = torch.empty(race.n, dtype=torch.float32, device=dev)
    _bbe.race_prefix(race, seed, request, sim, target, tick, pos, prev, state=state,
                     stream=stream)
    return tick, pos, prev


def rank_counts(orders: torch.Tensor, n: int, stream=None) -> torch.Tensor:
    """Finish-position counts [n, n] (int64, device) of an orders matrix:
    entry [c, r] = simulations in which competitor c finished at rank r."""
    counts = torch.empty((n, n), dtype=torch.int64, device=orders.device)
    _bbe.rank_counts(orders, n, counts, stream=stream)
    return counts


def order_pmf(orders: torch.Tensor, n: int, stream=None) -> torch.Tensor:
    """Counts [n!] (int64, device) of complete finish orders, indexed by the
    lexicographic rank of the permutation."""
    import math
    counts = torch.empty(math.factorial(n), dtype=torch.int64, device=orders.device)
    _bbe.order_pmf(orders, n, counts, stream=stream)
    return counts


def trace(race: Race, seed: int, request: int, sim: int, max_rows: int, state=None,
          stream=None, device=None):
    """Positions of one simulated race tick by tick.  Returns a float32 CUDA
    tensor [rows, n] (row 0 = the start state) -- synchronises to size it."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    buf = torch.empty((max_rows, race.n), dtype=torch.float32, device=dev)
    rows = torch.empty(1, dtype=torch.int32, device=dev)
    _bbe.race_trace(race, seed, request, sim, max_rows, buf, rows, state=state, stream=stream)
    return buf[: int(rows.item())]


def bettor_views(bettors, trace: torch.Tensor, track_len: float, t0: int, seed: int,
                 first_row: int = 0, n_eval: int | None = None, want_views: bool = True,
                 stream=None):
    """Views [n_eval, B] (uint8) and counts [n_eval, n] (int32) of a
    :class:`Bettors` population over rows of a trace tensor."""
    n_rows, n = trace.shape
    if n_eval is None:
        n_eval = n_rows - first_row
    views = (torch.empty((n_eval, bettors.n), dtype=torch.uint8, device=trace.device)
             if want_views else None)
    counts = torch.empty((n_eval, n), dtype=torch.int32, device=trace.device)
    bettors.views(trace, n_rows, track_len, t0, seed, first_row, n_eval, views=views,
                  counts=counts, stream=stream)
    return views, counts


def rp_views(wins: torch.Tensor, n: int, stream=None):
    """Views [B] (uint8) and counts [n] (int32) of RP(d) bettors from their
    win counts [B, stride] (int64)."""
    views = torch.empty(wins.shape[0], dtype=torch.uint8, device=wins.device)
    counts = torch.empty(n, dtype=torch.int32, device=wins.device)
    _bbe.rp_views(wins, n, views=views, counts=counts, stream=stream)
    return views, counts
