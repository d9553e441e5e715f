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


def _continuous_tick_laws(lo, hi, L, h, n_t, tol=1e-13):
    """Per tick k = 1, 2, ...: G_k on the fraction grid t_j = j / n_t
    (j = 0..n_t), G_k(t) = P(cross in tick k with fraction <= t), and
    S_k = P(not crossed after k ticks), for steps U(lo, hi) with a continuous
    uniform draw, in float64.

    The density of the position after k ticks (restricted to [0, L): a
    competitor at or past L has crossed) is carried on the grid y = i h,
    0 <= y <= L (its value at L the limit from below), and
    advanced by the box filter p_k(y) = (1/span) * integral of p_{k-1} over
    [y - hi, y - lo], using a cumulative trapezoid rule; the first two ticks
    are taken from their closed forms (uniform, then the trapezoid density
    of a sum of two uniforms) so that no jump of the density is integrated
    numerically.  lo, hi and L must be multiples of h."""
    span = hi - lo
    n = int(round(L / h)) + 1  # y = 0, h, ..., L: the density below the line
    y = np.arange(n) * h      # extended continuously to its end point L
    a, b = int(round(lo / h)), int(round(hi / h))
    t = np.arange(n_t + 1) / n_t

    def cross_law(p_prev):
        # G(t) = integral of p_prev(y) * P(x >= (L - y) / t) over y, for the
        # positions within one step of the line; trapezoid in y
        i0 = max(0, n - 1 - b)
        yy = y[i0:]
        pp = p_prev[i0:]
        w = np.full(len(yy), h)
        w[0] = w[-1] = h / 2
        rem = L - yy
        with np.errstate(divide="ignore", invalid="ignore"):
            need = rem[None, :] / t[:, None]  # the step x that crossing needs
        prob = np.clip((hi - need) / span, 0.0, 1.0)
        prob[0, :] = 0.0  # fraction 0: only a competitor exactly on the line
        return prob @ (w * pp)

    def box(p):
        c = np.concatenate([[0.0], np.cumsum((p[1:] + p[:-1]) * (h / 2))])
        idx_hi = np.arange(n) - a  # upper end of the window: y - lo
        idx_lo = np.arange(n) - b  # lower end: y - hi
        up = np.where(idx_hi >= 0, c[np.clip(idx_hi, 0, n - 1)], 0.0)
        dn = np.where(idx_lo >= 0, c[np.clip(idx_lo, 0, n - 1)], 0.0)
        return (up - dn) / span

    def mass(p):
        return float(np.sum((p[1:] + p[:-1]) * (h / 2)))

    if hi >= L:
        raise ValueError("a single step reaches the line")
    # G[k]: crossing in tick k, from the density after k - 1 ticks; S[k]:
    # survival after k ticks.  Tick 1 cannot cross; the densities after one
    # and two ticks are the uniform and the trapezoid of two uniforms.
    G = [np.zeros(n_t + 1), np.zeros(n_t + 1)]
    S = [1.0, 1.0]
    p_prev = np.where((y >= lo) & (y <= hi), 1.0 / span, 0.0)  # after tick 1
    G.append(cross_law(p_prev))
    p_cur = np.clip(np.minimum(y - 2 * lo, 2 * hi - y), 0.0, span) / (span * span)
    S.append(mass(p_cur))  # after tick 2 (below the line)
    while S[-1] > tol:
        G.append(cross_law(p_cur))
        p_cur = box(p_cur)
        S.append(mass(p_cur))
    return G, S


def p_first_wins_continuous(a, b, L, h=1.0 / 64, n_t=1000):
    """P(competitor 0 wins) for two non-interacting competitors whose steps
    are continuous uniforms U(a), U(b) (``(lo, hi)`` pairs): A wins if it
    crosses in an earlier tick, or in the same tick with the smaller
    crossing fraction (equal fractions have probability zero).  A
    numerical integration independent of the simulation code, accurate to
    about 1e-6 for the races used in the tests."""
    GA, SA = _continuous_tick_laws(a[0], a[1], L, h, n_t)
    GB, SB = _continuous_tick_laws(b[0], b[1], L, h, n_t)
    p = 0.0
    for k in range(1, len(GA)):
        ga = GA[k]
        pa_k = ga[-1]
        if pa_k == 0.0:
            continue
        sb_k = SB[k] if k < len(SB) else 0.0
        p += pa_k * sb_k
        if k < len(GB):
            gb = GB[k]
            # same tick: A's fraction below B's; midpoint rule on the t grid
            dga = np.diff(ga)
            gb_mid = 0.5 * (gb[1:] + gb[:-1])
            p += float(np.sum(dga * (gb[-1] - gb_mid)))
    return p
