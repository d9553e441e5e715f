"""Float64 reference of the surrogate network and of its encoder.

TEST INFRASTRUCTURE ONLY.  Shares no code with the GPU library.

Network: 160 -> 256 -> 256 -> 256 -> 20, ReLU after the three hidden
layers, softmax over the slots that hold a competitor (the others are
masked out), soft cross-entropy against Monte-Carlo win frequencies
(the frequentist estimates of paper Section 3), Adam (Kingma & Ba, 2015).

Parameters are one flat float32 vector packed as
  W1 [256,160], b1 [256], W2 [256,256], b2 [256], W3 [256,256], b3 [256],
  W4 [20,256], b4 [20]                                    (177,940 values)
with W[n, k] the weight from input k to output n.

Rounding points mirrored from the GPU kernels when ``bf16=True``: the
input features, the weights used in products, the hidden activations after
ReLU and the gradients fed to products (dz and the back-propagated
gradients) are rounded to bfloat16 (round to nearest even); everything else
is carried in float64 here (float32 on the GPU).  With ``bf16=False`` the
same formulas run in plain float64, which is what the finite-difference
check differentiates.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 160, 256, 20
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (OUT, HID)), ("b4", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, X, n_valid, bf16_on=True):
    """Logits [B, 20] (masked slots -inf), probabilities, and the cache."""
    P = unpack(params)
    x = _r(X, bf16_on)
    W = {k: _r(P[k], bf16_on) if k.startswith("W") else P[k] for k in P}
    a1 = x @ W["W1"].T + W["b1"]
    h1 = _r(np.maximum(a1, 0.0), bf16_on)
    a2 = h1 @ W["W2"].T + W["b2"]
    h2 = _r(np.maximum(a2, 0.0), bf16_on)
    a3 = h2 @ W["W3"].T + W["b3"]
    h3 = _r(np.maximum(a3, 0.0), bf16_on)
    z = h3 @ W["W4"].T + W["b4"]
    mask = np.arange(OUT)[None, :] < np.asarray(n_valid)[:, None]
    zm = np.where(mask, z, -np.inf)
    zmax = zm.max(axis=1, keepdims=True)
    e = np.where(mask, np.exp(zm - zmax), 0.0)
    q = e / e.sum(axis=1, keepdims=True)
    cache = dict(x=x, W=W, h1=h1, h2=h2, h3=h3, mask=mask)
    return zm, q, cache


def entropy(q):
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(q > 0, -q * np.log(q), 0.0)
    return t.sum(axis=1)


def loss_and_grad(params, X, n_valid, target, bf16_on=True):
    """Mean soft cross-entropy over the batch and its gradient (flat)."""
    B = X.shape[0]
    z, q, c = forward(params, X, n_valid, bf16_on)
    mask = c["mask"]
    with np.errstate(divide="ignore", invalid="ignore"):
        logq = np.where(mask, np.log(np.where(mask, q, 1.0)), 0.0)
    loss = -(np.asarray(target, np.float64) * logq).sum() / B
    dz = np.where(mask, (q - target) / B, 0.0)
    W = c["W"]
    g = {}
    d4 = _r(dz, bf16_on)
    g["W4"] = d4.T @ c["h3"]
    g["b4"] = d4.sum(axis=0)
    d3 = _r((d4 @ W["W4"]) * (c["h3"] > 0), bf16_on)
    g["W3"] = d3.T @ c["h2"]
    g["b3"] = d3.sum(axis=0)
    d2 = _r((d3 @ W["W3"]) * (c["h2"] > 0), bf16_on)
    g["W2"] = d2.T @ c["h1"]
    g["b2"] = d2.sum(axis=0)
    d1 = _r((d2 @ W["W2"]) * (c["h1"] > 0), bf16_on)
    g["W1"] = d1.T @ c["x"]
    g["b1"] = d1.sum(axis=0)
    return loss, pack(g)


# ---------------------------------------------------------------------------
# Per-element bounds for checking one layer of a float32-accumulating
# implementation on its own inputs.
#
# A sum of m terms evaluated in float32 in any order, each addition one
# rounding, differs from the exact sum by at most gamma_m * sum|t| with
# gamma_m = m*u / (1 - m*u) (Higham, "Accuracy and Stability of Numerical
# Algorithms", 2nd ed., Lemma 3.1 and Eq. 3.5).  u is taken as 2^-23, one
# unit in the last place rather than half of one, so that adders that
# truncate are covered too.  Products of two bfloat16 values are exact in
# float32 (8 + 8 significant bits), so the sum is the only error source.
# The float64 evaluation of the exact sum adds at most m * 2^-53 * sum|t|,
# which is added to the bound.
# ---------------------------------------------------------------------------
U_F32 = 2.0 ** -23


def accumulation_bound(abs_sum, m):
    """Bound on |float32 sum - exact sum| for m terms with sum|t| = abs_sum."""
    m = float(m)
    g = m * U_F32 / (1.0 - m * U_F32) + m * 2.0 ** -53
    return g * np.asarray(abs_sum, dtype=np.float64)


def dense_with_bound(h, W, b=None):
    """Pre-activation h @ bf16(W)^T (+ b) in float64 and the bound on the
    error of computing it with float32 accumulation (the bias, when given,
    is one more term of the sum).  h must already be bfloat16 values."""
    Wb = bf16(W)
    h = np.asarray(h, dtype=np.float64)
    a = h @ Wb.T
    abs_sum = np.abs(h) @ np.abs(Wb).T
    m = h.shape[1]
    if b is not None:
        a = a + np.asarray(b, dtype=np.float64)
        abs_sum = abs_sum + np.abs(np.asarray(b, dtype=np.float64))
        m += 1
    return a, accumulation_bound(abs_sum, m)


def bf16_interval(a, e, relu=False):
    """The bfloat16 values that rounding any float in [a - e, a + e] (after
    ReLU when relu=True) can give lie in the returned [lo, hi]: rounding to
    nearest and ReLU are both non-decreasing."""
    lo, hi = np.asarray(a) - e, np.asarray(a) + e
    if relu:
        lo, hi = np.maximum(lo, 0.0), np.maximum(hi, 0.0)
    return bf16(lo), bf16(hi)


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) -> (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def encode(comp, n, pos, prev, track_len, dt):
    """Features [B, 160] (float32, before bfloat16 rounding) and the
    competitor index in each slot [B, 20] (-1 for padding).

    Slots hold the competitors by expected remaining ticks T (below),
    smallest first (equal T: lower index first), padded to 20: early in a
    race that orders the field by strength, late in it by position.
    Positions enter only as distances relative to other competitors or to
    the line, so that bfloat16 keeps the gaps that decide a race.  Per slot
    8 features, each one float32 operation sequence (v = fl(7.5 dt),
    w = fl(75 dt), c15 = fl(15 dt)):
      1 rem  = (L-d)/L                       remaining distance
      2 lead = (d_lead - d)/w                gap to the leader on the track
      3 gap  = min((d_up - d)/v, 4)          gap to the competitor directly ahead on
                                             the track (position order, equal
                                             positions by index; 4 for the leader)
      4 s/v                                  previous step
      5 spd  = (lo+hi)/c15                   mean free step over 7.5 dt
      6 (hi-lo)/(hi+lo)                      relative noise
      7 rho/0.2                              responsiveness
      8 (T - T_min)/10                       expected remaining ticks behind the best
    with T = (L-d) / ((lo+hi)*0.5 * (1 + rho*(d/L))): the remaining distance
    at the mean free step scaled by R_c at the midpoint of the remaining
    distance (1 + rho*(2*((L+d)/2)/L - 1) = 1 + rho*d/L), and T_min the
    smallest T of the state.  Padding slots are 0."""
    f = np.float32
    comp = np.asarray(comp, np.float32)
    B = comp.shape[0]
    L = f(track_len)
    v = f(f(7.5) * f(dt))
    w = f(f(75.0) * f(dt))
    c15 = f(f(15.0) * f(dt))
    X = np.zeros((B, 20, 8), dtype=np.float32)
    slot = np.full((B, 20), -1, dtype=np.int32)
    for b in range(B):
        k = int(n[b])
        by_pos = sorted(range(k), key=lambda c: (-float(pos[b][c]), c))  # the track, leader first
        T = []
        for c in range(k):
            lo, hi, _, rho, _ = comp[b, c]
            d = f(pos[b][c])
            rmid = f(f(1.0) + f(rho * f(d / L)))
            T.append(f(f(L - d) / f(f(f(lo + hi) * f(0.5)) * rmid)))
        order = sorted(range(k), key=lambda c: (float(T[c]), c))
        t_min = min(T) if T else f(0.0)
        d_lead = f(pos[b][by_pos[0]]) if k else f(0.0)
        for r, c in enumerate(order):
            lo, hi, _, rho, _ = comp[b, c]
            d, s = f(pos[b][c]), f(prev[b][c])
            q = by_pos.index(c)  # its place on the track
            gap = f(4.0) if q == 0 else min(f(f(f(pos[b][by_pos[q - 1]]) - d) / v), f(4.0))
            X[b, r] = [f(f(L - d) / L), f(f(d_lead - d) / w), gap, f(s / v),
                       f(f(lo + hi) / c15), f(f(hi - lo) / f(hi + lo)), f(rho / f(0.2)),
                       f(f(T[c] - t_min) / f(10.0))]
            slot[b, r] = c
    return X.reshape(B, 160), slot
