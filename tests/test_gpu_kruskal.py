"""Cross-implementation comparison in the paper's way (Section 6: the PMFs
over finish orders that repeated runs with different seeds estimate are
compared with a Kruskal-Wallis test, to tell noise from consistent
variation): the GPU library and the CPU oracle, run with different seeds,
give finish-order and finishing-position samples that the test cannot
tell apart, while a race with one competitor 3% faster is told apart."""
import math

import numpy as np
import pytest
from scipy import stats

from gpu_util import announce, require_gpu
from oracle import orders as O
from paper_2108_02419_amd import api, inputs
from paper_2108_02419_amd._bbe import Race

pytestmark = pytest.mark.gpu

N = 100_000
L = inputs.TRACK_LEN


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _gpu_samples(torch, comp, seed):
    """Finish-order indices (from the device PMF counts) and the finishing
    position of every competitor, N simulations from the start."""
    n = comp.shape[0]
    race = Race(comp, L)
    out = api.mc(race, N, seed, request=1, want_orders=True)
    pmf = api.order_pmf(out["orders"], n)
    torch.cuda.synchronize()
    counts = pmf.cpu().numpy().astype(np.int64)
    assert counts.sum() == N and counts.size == math.factorial(n)
    orders = out["orders"].cpu().numpy()
    pos = np.argsort(orders, axis=1)  # pos[s, c] = finishing position of competitor c
    return np.repeat(np.arange(counts.size), counts), pos


def _oracle_samples(orc, comp, seed):
    orders, _, _ = orc.race_sim(comp, L, N, seed, request=1, threads=8)
    return np.array([O.lex_rank(r) for r in orders]), np.argsort(orders, axis=1)


def test_gpu_and_oracle_outcomes_are_indistinguishable(torch, orc):
    comp = inputs.competitor_params(np.random.default_rng(1), 5)
    announce("Kruskal-Wallis: GPU seed 101 vs GPU seed 202 vs oracle seed 303")
    g1_idx, g1_pos = _gpu_samples(torch, comp, 101)
    g2_idx, g2_pos = _gpu_samples(torch, comp, 202)
    o_idx, o_pos = _oracle_samples(orc, comp, 303)
    p = stats.kruskal(g1_idx, g2_idx, o_idx).pvalue
    assert p > 1e-3, p
    for c in range(comp.shape[0]):
        pc = stats.kruskal(g1_pos[:, c], g2_pos[:, c], o_pos[:, c]).pvalue
        assert pc > 1e-4, (c, pc)  # five tests: a family-wise level of 5e-4


def test_a_faster_competitor_is_told_apart(torch, orc):
    comp = inputs.competitor_params(np.random.default_rng(1), 5)
    faster = comp.copy()
    faster[2, :2] *= np.float32(1.03)  # competitor 2 steps 3% further
    announce("Kruskal-Wallis: a competitor 3% faster")
    _, g_pos = _gpu_samples(torch, comp, 101)
    _, f_pos = _gpu_samples(torch, faster, 202)
    assert stats.kruskal(g_pos[:, 2], f_pos[:, 2]).pvalue < 1e-6
