"""How much the resolution of the uniform draw matters (a reading of paper
Section 3, where the stochastic step is U(lo, hi) with no stated
resolution): the draw is read as a 16-bit fraction k / 2^16.  Coarsening it
sixteen-fold, to 2^12 levels, must leave the finish-order distribution of
the five-competitor start workload unchanged within Monte-Carlo noise at
10^6 simulations per side; a 16-bit draw is closer still to a continuous
one than a 12-bit draw is to a 16-bit one."""
import os

import numpy as np
import pytest

from paper_2108_02419_amd import inputs

N_SIMS = 1_000_000


def _pmf(orders):
    """Counts of each complete finish order (rows as bytes)."""
    keys, counts = np.unique(np.ascontiguousarray(orders).view(np.dtype((np.void, orders.shape[1]))),
                             return_counts=True)
    return {bytes(k): int(c) for k, c in zip(keys, counts)}


@pytest.mark.slow
def test_finish_order_pmf_insensitive_to_draw_resolution(orc):
    c = inputs.start_config(inputs.CFG_START_N5)
    threads = max(1, min(8, os.cpu_count() or 1))
    # independent streams (different seeds), so each side's noise is its own
    fine, _, _ = orc.race_sim(c["comp"], c["L"], N_SIMS, 1, threads=threads)
    coarse, _, _ = orc.race_sim(c["comp"], c["L"], N_SIMS, 1001, levels=1 << 12, threads=threads)
    a, b = _pmf(fine), _pmf(coarse)
    assert sum(a.values()) == sum(b.values()) == N_SIMS
    keys = sorted(set(a) | set(b))
    pa = np.array([a.get(k, 0) for k in keys], np.float64) / N_SIMS
    pb = np.array([b.get(k, 0) for k in keys], np.float64) / N_SIMS
    pbar = 0.5 * (pa + pb)
    sigma = np.sqrt(np.maximum(pbar * (1 - pbar), 1.0 / N_SIMS) * 2.0 / N_SIMS)
    z = np.abs(pa - pb) / sigma
    assert z.max() < 5.0, (float(z.max()), keys[int(z.argmax())])
    # the whole distribution: chi-square homogeneity over orders seen >= 50 times
    from scipy import stats
    m = (pa + pb) * N_SIMS >= 50
    table = np.stack([pa[m], pb[m]]) * N_SIMS
    _, p, _, _ = stats.chi2_contingency(table)
    assert p > 1e-4, p
    # paired view on one stream: the coarse draw changes few finish orders
    same_seed, _, _ = orc.race_sim(c["comp"], c["L"], 100_000, 1, levels=1 << 12,
                                   threads=threads)
    changed = (same_seed != fine[:100_000]).any(axis=1).mean()
    assert changed < 0.2, changed
