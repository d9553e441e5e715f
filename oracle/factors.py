"""Preference coefficient from race factors, written out plainly (paper
Section 3: P_c(f_r, p_c) in [0, 1] scales a competitor's stochastic step
down by an amount that grows with the mismatch between the race's factors
f_r and the competitor's preferred values p_c).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing in the
product library.

Reading (the paper gives no formula; its companion paper is not
available): factors and preferences are normalised to [0, 1], so the
mismatch on factor k is |f_k - p_ck| in [0, 1]; each competitor has a
sensitivity w_ck in [0, 1) per factor; each factor scales the step by
1 - w_ck * |f_k - p_ck| independently of the others, so

    P_c = prod_k (1 - w_ck * |f_k - p_ck|),

in single precision, one rounding per operation, factors taken in order
k = 0, 1, ...  Every term is at least 1 - w_ck > 0; a product that
underflows to 0 is rejected (the step would vanish).
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def pref_from_factors(f, p, w) -> np.ndarray:
    """P [n] (float32) from factors f [F], preferences p [n, F] and
    sensitivities w [n, F]."""
    f = np.asarray(f, dtype=np.float32)
    p = np.asarray(p, dtype=np.float32)
    w = np.asarray(w, dtype=np.float32)
    n, F = p.shape
    out = np.zeros(n, dtype=np.float32)
    for c in range(n):
        P = f32(1.0)
        for k in range(F):
            mismatch = abs(f32(f[k] - p[c, k]))
            P = f32(P * f32(f32(1.0) - f32(w[c, k] * mismatch)))
        if not P > 0:
            raise ValueError(f"competitor {c}: P underflows to 0")
        out[c] = P
    return out
