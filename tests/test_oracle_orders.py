"""Pins of the finish-order tallies (oracle/orders.py): the lexicographic
index against an independent enumeration of permutations, hand-worked
counts, and the order PMF against the exact PMF of tiny races."""
import itertools

import numpy as np
import pytest

from oracle import orders as O
from oracle.enumerate import enumerate_race


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_lex_rank_is_the_index_in_sorted_permutations(n):
    for k, perm in enumerate(sorted(itertools.permutations(range(n)))):
        assert O.lex_rank(perm) == k


def test_rank_counts_and_pmf_by_hand():
    rows = np.array([[2, 0, 1], [0, 1, 2], [2, 1, 0xFF], [2, 0, 1]], np.uint8)
    want = np.zeros((3, 3), np.uint64)
    # rank 0: 2, 0, 2, 2; rank 1: 0, 1, 1, 0; rank 2: 1, 2, -, 1
    want[2, 0], want[0, 0] = 3, 1
    want[0, 1], want[1, 1] = 2, 2
    want[1, 2], want[2, 2] = 2, 1
    np.testing.assert_array_equal(O.rank_counts(rows, 3), want)
    pmf = O.order_pmf(rows, 3)
    # (0,1,2) is permutation 0, (2,0,1) is permutation 4; the partial row is skipped
    assert pmf.tolist() == [1, 0, 0, 0, 2, 0]


def test_order_pmf_matches_exact_pmf(orc):
    comp = np.array([[1, 2, 1, 0, 0.5], [1, 2, 1, 0.2, 0.5], [1, 2, 1, -0.2, 0]], np.float32)
    K, L, N = 2, 4.0, 100_000
    pmf, _ = enumerate_race(comp, L, K, stop_after=3)
    orders, _, _ = orc.race_sim(comp, L, N, seed=77, levels=K, stop_after=3, threads=8)
    counts = O.order_pmf(orders, 3)
    assert int(counts.sum()) == N
    for order, p in pmf.items():
        p = float(p)
        got = counts[O.lex_rank(order)] / N
        assert abs(got - p) <= 5 * np.sqrt(p * (1 - p) / N) + 1e-12, (order, got, p)
    rc = O.rank_counts(orders, 3)
    assert (rc.sum(axis=0) == N).all() and (rc.sum(axis=1) == N).all()
