"""Full-length two-competitor races: oracle Monte-Carlo against the exact law
from oracle/twocomp.py (no interaction: theta = 0, rho = 0).  The first case
is the paper's own example pair of step laws U(10,20) and U(1,25)
(Section 3) on a 2000-unit track."""
import numpy as np
import pytest

from oracle.twocomp import p_first_wins

CASES = [
    ("paper_example_U10_20_vs_U1_25", (10.0, 20.0), (1.0, 25.0), 8),
    ("close_race_U10_20_vs_U11_19", (10.0, 20.0), (11.0, 19.0), 8),
    ("short_track_U1_2_vs_U1_3", (1.0, 2.0), (1.0, 3.0), 4),
]


@pytest.mark.parametrize("name,a,b,K", CASES, ids=[c[0] for c in CASES])
def test_two_competitor_law(orc, name, a, b, K):
    L = 2000.0 if a[0] >= 10 else 40.0
    p = p_first_wins(a, b, L, K)
    comp = np.array([[a[0], a[1], 1, 0, 0], [b[0], b[1], 1, 0, 0]], np.float32)
    N = 1_000_000
    _, wins, _ = orc.race_sim(comp, L, N, seed=11, stop_after=1, levels=K, want_orders=False,
                              threads=8)
    assert wins.sum() == N
    ph = wins[0] / N
    sig = np.sqrt(max(p * (1 - p), 1.0 / N) / N)
    assert abs(ph - p) <= 5 * sig, (ph, p, sig)


def test_continuous_law_symmetry_and_complement():
    """The continuous winner law (a numerical integration apart from the
    simulation code): equal step laws give 1/2, and swapping the two
    competitors gives the complement (equal fractions have probability 0)."""
    from oracle.twocomp import p_first_wins_continuous
    assert abs(p_first_wins_continuous((10.0, 20.0), (10.0, 20.0), 2000.0) - 0.5) < 1e-6
    ab = p_first_wins_continuous((10.0, 20.0), (11.0, 19.0), 2000.0)
    ba = p_first_wins_continuous((11.0, 19.0), (10.0, 20.0), 2000.0)
    assert abs(ab + ba - 1.0) < 1e-6


@pytest.mark.parametrize("a,b", [((10.0, 20.0), (1.0, 25.0)), ((10.0, 20.0), (11.0, 19.0))],
                         ids=["paper_example", "close_race"])
def test_oracle_with_16_bit_draws_against_continuous_law(orc, a, b):
    """The oracle's own draw resolution (16 bits, levels = 0) against the
    continuous law at 10^6 simulations, within 5 sigma."""
    from oracle.twocomp import p_first_wins_continuous
    L = 2000.0
    p = p_first_wins_continuous(a, b, L)
    comp = np.array([[a[0], a[1], 1, 0, 0], [b[0], b[1], 1, 0, 0]], np.float32)
    N = 1_000_000
    _, wins, _ = orc.race_sim(comp, L, N, seed=12, stop_after=1, want_orders=False, threads=8)
    sig = np.sqrt(max(p * (1 - p), 1.0 / N) / N)
    assert abs(wins[0] / N - p) <= 5 * sig, (wins[0] / N, p, sig)
