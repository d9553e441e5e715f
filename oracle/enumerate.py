"""Exact enumeration of tiny races -- an independent implementation of the
race model (paper Section 3, Eq. 1) in plain Python with numpy float32
scalars.

TEST INFRASTRUCTURE ONLY.  It shares no code with the C oracle or the GPU
library; it exists to pin the C oracle.

Draws are restricted to K equally spaced levels u in {0, 1/K, ..., (K-1)/K}.
Every draw sequence a race can consume is enumerated (only competitors that
are not blocked consume a draw), so the exact probability mass function over
finish orders follows, each path weighing K^-(draws consumed) -- the PMF the
paper estimates by repeated seeded runs (Section 6).  Each path is also
returned with the draws it consumed, so that the C oracle can be driven with
the same draws and must reproduce the same order.

Single-precision operation order (one rounding per operation):
  elo = P*lo, espan = P*(hi-lo), alpha = 1-rho, beta = (2*rho)/L  (set-up)
  R = (alpha + beta*d_c) + gamma*min(t, tau)  (t the absolute tick; rows of
      5 parameters mean gamma = 0);  unblocked: S = R*(elo + espan*u);
  blocked: S = R*min(s_c, s_ahead);  crossing fraction (L - d_old)/S.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product

import numpy as np

f32 = np.float32


class Race:
    def __init__(self, comp, L):
        comp = np.asarray(comp, dtype=np.float32)
        self.n = comp.shape[0]
        self.L = f32(L)
        self.elo, self.espan, self.alpha, self.beta, self.theta = [], [], [], [], []
        self.gamma, self.tau = [], []
        for row in comp:
            lo, hi, pref, rho, theta = (f32(v) for v in row[:5])
            gamma, tau = (f32(row[5]), f32(row[6])) if len(row) == 7 else (f32(0), f32(0))
            self.gamma.append(gamma)
            self.tau.append(tau)
            self.elo.append(f32(pref * lo))
            self.espan.append(f32(pref * f32(hi - lo)))
            self.alpha.append(f32(f32(1.0) - rho))
            self.beta.append(f32(f32(f32(2.0) * rho) / self.L))
            self.theta.append(theta)


def _ahead(race, d, s, running, c):
    """(gap, previous step) of the nearest running competitor strictly ahead of
    c -- the smallest position greater than d_c, the lowest index among equal
    positions; (inf, None) when nobody is ahead."""
    cands = [i for i in running if i != c and d[i] > d[c]]
    if not cands:
        return f32(np.inf), None
    i = min(cands, key=lambda i: (d[i], i))
    return f32(d[i] - d[c]), s[i]


def enumerate_race(comp, L, K, stop_after=None, state=None, max_ticks=64):
    """Exact PMF over finish orders for draws restricted to K levels.

    Returns ``(pmf, paths)``: ``pmf`` maps an order (tuple of competitor ids,
    unranked ones omitted) to a Fraction; ``paths`` is a list of
    ``(consumed, order, prob, trace)`` where ``consumed`` maps (relative tick,
    competitor) to the level index drawn and ``trace`` lists the positions
    after every tick.
    """
    race = Race(comp, L)
    n = race.n
    stop_after = n if stop_after is None else stop_after
    t0 = 0 if state is None else int(state[0])
    if state is None:
        d0 = [f32(0.0)] * n
        s0 = [f32(0.0)] * n
    else:
        d0 = [f32(x) for x in state[1]]
        s0 = [f32(x) for x in state[2]]
    levels = [f32(j) / f32(K) for j in range(K)]
    pmf: dict[tuple, Fraction] = {}
    paths = []

    def rec(tick, d, s, running, order, prob, consumed, trace):
        if len(order) >= stop_after:
            key = tuple(order)
            pmf[key] = pmf.get(key, Fraction(0)) + prob
            paths.append((dict(consumed), key, prob, list(trace)))
            return
        if tick >= max_ticks:
            raise RuntimeError("race did not finish within max_ticks")
        # Eq. 1, first part: who is blocked, from the start-of-tick state.
        plan = {}
        for c in sorted(running):
            gap, s_ahead = _ahead(race, d, s, running, c)
            th = min(f32(t0 + tick), race.tau[c])
            R = f32(f32(race.alpha[c] + f32(race.beta[c] * d[c])) + f32(race.gamma[c] * th))
            if gap > race.theta[c]:
                plan[c] = ("free", R, None)
            else:
                plan[c] = ("blocked", R, f32(R * min(s[c], s_ahead)))
        free = [c for c in sorted(running) if plan[c][0] == "free"]
        for combo in product(range(K), repeat=len(free)):
            draw = dict(zip(free, combo))
            S = {}
            for c in sorted(running):
                kind, R, Sb = plan[c]
                if kind == "free":
                    x = f32(race.elo[c] + f32(race.espan[c] * levels[draw[c]]))
                    S[c] = f32(R * x)
                else:
                    S[c] = Sb
            nd, ns = list(d), list(s)
            crossers = []
            for c in sorted(running):
                dn = f32(d[c] + S[c])
                if dn >= race.L:
                    crossers.append((f32(f32(race.L - d[c]) / S[c]), c))
                nd[c] = dn
                ns[c] = S[c]
            crossers.sort()  # by fraction, then index
            new_order = order + [c for _, c in crossers]
            new_running = running - {c for _, c in crossers}
            new_consumed = dict(consumed)
            for c, j in draw.items():
                new_consumed[(tick, c)] = j
            rec(tick + 1, nd, ns, new_running, new_order,
                prob / (K ** len(free)), new_consumed, trace + [list(nd)])

    rec(0, d0, s0, frozenset(range(n)), [], Fraction(1), {}, [])
    return pmf, paths


def draws_matrix(paths, n, K, n_ticks):
    """Dense [n_paths, n_ticks, n] float32 draw matrices (unused slots hold 0)."""
    out = np.zeros((len(paths), n_ticks, n), dtype=np.float32)
    for p, (consumed, _, _, _) in enumerate(paths):
        for (t, c), j in consumed.items():
            out[p, t, c] = np.float32(j) / np.float32(K)
    return out
