"""Cheap in-play bettor rules, written out plainly (paper Section 5).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing in the
product library.

Each bettor holds a view of which competitor will win, formed from the
race as it has unfolded so far.  The race is given as a trace: row r holds
the positions of the n competitors after r ticks from the trace's first
tick t0 (row 0 is the state at t0).  Four rules of Section 5:

  LW    (Leader Wins)  the competitor currently in the lead.
  UD    (Underdog, threshold D)  the second-placed competitor while its
        distance to the leader is below D, else the leader.
  LinEx (Linear Extrapolator, window N)  estimates each competitor's speed
        as its mean step over the last N ticks, assumes that speed holds
        to the line, and picks the competitor that would reach it first.
  ZI    (Zero Intelligence)  a competitor chosen uniformly at random.

and the view of an RP(d) bettor (Section 3), formed from its own dry-run
win counts: the competitor that won most of them.

Readings of points Section 5 leaves open:
  * Ties in position go to the lowest competitor index, for the leader
    and for the second-placed competitor alike.
  * UD's distance is fl(x_P1 - x_P2) in single precision; the view is P2
    iff that distance is strictly below D.  With one competitor UD is LW.
  * LinEx uses a window of w = min(N, r) ticks (the trace cannot look
    further back than its first row); with w = 0 it holds LW's view.  The
    mean step is disp_c / w with disp_c = fl(x_c(r) - x_c(r - w)), and the
    time to the line is fl(L - x_c(r)) / (disp_c / w); w is common to all
    competitors, so the pick minimises the exact ratio
    fl(L - x_c) / disp_c over the competitors with disp_c > 0 (exact
    rational comparison of the single-precision operands; equal ratios go
    to the lowest index).  If no competitor moved in the window LinEx
    holds LW's view.
  * An RP(d) bettor's view is the competitor with the most wins among its
    dry-runs, ties (and a bettor with no recorded win) to the lowest index.
  * ZI draws afresh at every tick: one Philox4x32-10 block with key
    (seed_lo, seed_hi) and counter (t, bettor, 0xffffffff, 0xffffffff);
    its first word w gives the competitor floor(w * n / 2^32).  The last
    counter word of a race draw is c >> 3 <= 2, so ZI draws never reuse a
    race draw even under the same key.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import philox4x32_10

ZI, LW, UD, LINEX = 0, 1, 2, 3
KINDS = {"ZI": ZI, "LW": LW, "UD": UD, "LinEx": LINEX}


def leader(x) -> int:
    """Index of the largest position, lowest index among equals."""
    best = 0
    for c in range(1, len(x)):
        if x[c] > x[best]:
            best = c
    return best


def second(x, p1: int) -> int:
    """Index of the largest position other than ``p1`` (lowest index among
    equals); ``x`` must have at least two entries."""
    best = -1
    for c in range(len(x)):
        if c == p1:
            continue
        if best < 0 or x[c] > x[best]:
            best = c
    return best


def zi_pick(seed: int, t: int, bettor: int, n: int) -> int:
    w = int(philox4x32_10([t & 0xFFFFFFFF, bettor, 0xFFFFFFFF, 0xFFFFFFFF],
                          [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])[0])
    return (w * n) >> 32


def linex_pick(trace, r: int, N: int, L: float) -> int:
    x = trace[r]
    w = min(N, r)
    if w == 0:
        return leader(x)
    back = trace[r - w]
    best, best_q = -1, None
    for c in range(len(x)):
        disp = np.float32(x[c]) - np.float32(back[c])
        if not disp > 0:
            continue
        rem = np.float32(L) - np.float32(x[c])
        q = Fraction(float(rem)) / Fraction(float(disp))
        if best < 0 or q < best_q:
            best, best_q = c, q
    return leader(x) if best < 0 else best


def view(kind: int, param: float, trace, r: int, L: float, t0: int, bettor: int,
         seed: int) -> int:
    """The view of one bettor at trace row ``r`` (tick t0 + r)."""
    x = np.asarray(trace[r], dtype=np.float32)
    n = len(x)
    if kind == ZI:
        return zi_pick(seed, t0 + r, bettor, n)
    if kind == LW:
        return leader(x)
    if kind == UD:
        p1 = leader(x)
        if n == 1:
            return p1
        p2 = second(x, p1)
        gap = np.float32(x[p1]) - np.float32(x[p2])
        return p2 if gap < np.float32(param) else p1
    if kind == LINEX:
        return linex_pick(np.asarray(trace, dtype=np.float32), r, int(param), L)
    raise ValueError(f"unknown bettor kind {kind}")


def views(kinds, params, trace, L: float, t0: int, seed: int, first_row: int = 0,
          n_eval: int | None = None):
    """Views ``[n_eval, B]`` (uint8) and view counts ``[n_eval, n]`` (uint32)
    of the bettors at trace rows first_row .. first_row + n_eval - 1."""
    trace = np.asarray(trace, dtype=np.float32)
    rows, n = trace.shape
    if n_eval is None:
        n_eval = rows - first_row
    B = len(kinds)
    out = np.zeros((n_eval, B), dtype=np.uint8)
    counts = np.zeros((n_eval, n), dtype=np.uint32)
    for i in range(n_eval):
        r = first_row + i
        for b in range(B):
            v = view(int(kinds[b]), float(params[b]), trace, r, L, t0, b, seed)
            out[i, b] = v
            counts[i, v] += 1
    return out, counts


def rp_views(wins, n: int):
    """Views ``[B]`` (uint8) and view counts ``[n]`` (uint32) of RP(d)
    bettors from their win counts ``[B, >= n]`` (competitors 0..n-1)."""
    wins = np.asarray(wins)
    B = wins.shape[0]
    out = np.zeros(B, dtype=np.uint8)
    counts = np.zeros(n, dtype=np.uint32)
    for b in range(B):
        best = 0
        for c in range(1, n):
            if int(wins[b, c]) > int(wins[b, best]):
                best = c
        out[b] = best
        counts[best] += 1
    return out, counts
