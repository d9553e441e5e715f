"""Exact winner law of a two-competitor race without interaction.

TEST INFRASTRUCTURE ONLY -- pins the C oracle on full-length races.

With theta = 0 nobody is ever blocked (the gap to a competitor ahead is
always > 0) and with rho = 0 the responsiveness is 1, so by Eq. 1 each
competitor's position is a plain sum of independent steps
elo + espan*u (paper Section 3: d_c(t+dt) = d_c(t) + S_c(t)).  With u on K
levels the law of each competitor's crossing tick and crossing fraction
follows from a dynamic program over positions, and the winner law from the
two independent laws: A wins if it crosses in an earlier tick, or in the
same tick with a smaller or equal fraction (A has the lower index).

Positions are carried in float32, one rounding per addition, exactly as the
model prescribes; probabilities in float64.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

f32 = np.float32


def crossing_law(lo, hi, L, K, max_ticks=100_000):
    """Law of (crossing tick, crossing fraction) from the start line.

    Returns ``(cross, survive)``: ``cross[k]`` is a dict fraction -> prob for
    crossing in tick k (1-based), ``survive[k]`` = P(not crossed after k
    ticks), with ``survive[0] = 1``.
    """
    lo, hi, L = f32(lo), f32(hi), f32(L)
    elo = f32(f32(1.0) * lo)
    espan = f32(f32(1.0) * f32(hi - lo))
    steps = [f32(elo + f32(espan * f32(f32(j) / f32(K)))) for j in range(K)]
    p_step = 1.0 / K
    dist = {f32(0.0): 1.0}
    cross = [dict()]
    survive = [1.0]
    k = 0
    while dist:
        k += 1
        if k > max_ticks:
            raise RuntimeError("race too long")
        nxt = defaultdict(float)
        here = defaultdict(float)
        for y, p in dist.items():
            rem = f32(L - y)
            for x in steps:
                dn = f32(y + x)
                if dn >= L:
                    here[f32(rem / x)] += p * p_step
                else:
                    nxt[dn] += p * p_step
        cross.append(dict(here))
        dist = dict(nxt)
        survive.append(float(sum(dist.values())))
    return cross, survive


def p_first_wins(a, b, L, K):
    """P(competitor 0 wins) for two non-interacting competitors with step laws
    U(a) and U(b) (``(lo, hi)`` pairs) on K draw levels."""
    ca, sa = crossing_law(a[0], a[1], L, K)
    cb, sb = crossing_law(b[0], b[1], L, K)
    p = 0.0
    for k in range(1, len(ca)):
        if not ca[k]:
            continue
        pa_k = sum(ca[k].values())
        later_b = sb[k] if k < len(sb) else 0.0
        p += pa_k * later_b
        if k < len(cb) and cb[k]:
            fb = np.array(sorted(cb[k].keys()), dtype=np.float32)
            pb = np.array([cb[k][f] for f in fb])
            tail = np.cumsum(pb[::-1])[::-1]  # P(B frac >= fb[i])
            for fa, pa in ca[k].items():
                i = int(np.searchsorted(fb, fa, side="left"))
                if i < len(fb):
                    p += pa * tail[i]
    return p
