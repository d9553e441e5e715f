"""Test infrastructure (CPU oracle): tallies over finish orders, written from
their definitions (paper Section 6: the finish orders of repeated runs
estimate a PMF over the n! orders).  Only tests, smoke() and the CPU baseline
use this module."""
from __future__ import annotations

import math

import numpy as np

UNRANKED = 0xFF


def rank_counts(orders, n: int) -> np.ndarray:
    """counts[c, r] = number of rows whose rank r holds competitor c
    (unranked places skipped)."""
    orders = np.asarray(orders, dtype=np.uint8).reshape(-1, n)
    counts = np.zeros((n, n), dtype=np.uint64)
    for row in orders:
        for r, c in enumerate(row):
            if c < n:
                counts[c, r] += 1
    return counts


def lex_rank(order) -> int:
    """Position of a permutation of 0..n-1 in lexicographic order: for each
    place, the number of later entries smaller than it, weighted by the
    factorial of the number of places after it."""
    order = [int(v) for v in order]
    n = len(order)
    rank = 0
    for i, v in enumerate(order):
        smaller = sum(1 for w in order[i + 1:] if w < v)
        rank += smaller * math.factorial(n - 1 - i)
    return rank


def order_pmf(orders, n: int) -> np.ndarray:
    """counts[k] = number of complete rows equal to the k-th permutation in
    lexicographic order (rows with an unranked place skipped)."""
    orders = np.asarray(orders, dtype=np.uint8).reshape(-1, n)
    counts = np.zeros(math.factorial(n), dtype=np.uint64)
    for row in orders:
        if (row < n).all():
            counts[lex_rank(row)] += 1
    return counts
