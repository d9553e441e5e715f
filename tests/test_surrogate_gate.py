"""Host logic of the surrogate's Monte-Carlo fallback gate (no GPU)."""
import numpy as np
import torch

from paper_2108_02419_amd import surrogate as S


def _t(a):
    return torch.tensor(np.asarray(a))


def test_gate_is_the_last_entropy_before_the_first_miss():
    ref = np.zeros((5, 20)); ref[:, 0] = 1.0
    pred = ref.copy()
    # per-state max errors 0.00, 0.01, 0.05, 0.00, 0.03 ; entropies 0.1 .. 0.5 (shuffled)
    for i, e in enumerate([0.0, 0.01, 0.05, 0.0, 0.03]):
        pred[i, 0] -= e
        pred[i, 1] += e
    ent = np.array([0.2, 0.1, 0.4, 0.3, 0.5])
    n = np.full(5, 3)
    gate = S.calibrate_gate(_t(pred), _t(ent), _t(ref), _t(n), 0.02)
    # by entropy: 0.1 (err .01), 0.2 (0), 0.3 (0), 0.4 (.05 -> miss)
    assert gate == 0.3
    assert S.calibrate_gate(_t(pred), _t(ent), _t(ref), _t(n), 0.1) == 0.5
    worst_first = ent.copy(); worst_first[2] = 0.0
    assert S.calibrate_gate(_t(pred), _t(worst_first), _t(ref), _t(n), 0.02) == -1.0


def test_gated_errors_mix_surrogate_and_monte_carlo_answers():
    ref = np.zeros((4, 20)); ref[:, :2] = 0.5
    pred = ref.copy(); pred[:, 0] += [0.01, 0.2, 0.0, 0.3]; pred[:, 1] -= [0.01, 0.2, 0.0, 0.3]
    mc = ref.copy(); mc[:, 0] += 0.004; mc[:, 1] -= 0.004
    ent = np.array([0.1, 0.9, 0.2, 0.8])
    n = np.full(4, 2)
    g = S.gated_errors(_t(pred), _t(ent), _t(mc), _t(ref), _t(n), 0.5)
    assert g["served_frac"] == 0.5
    assert abs(g["served_max_err"] - 0.01) < 1e-12
    assert abs(g["answer_max_err"] - 0.01) < 1e-12
    assert abs(g["surrogate_max_err"] - 0.3) < 1e-12
    # padding slots never count
    pred2 = pred.copy(); pred2[:, 5] = 0.9
    assert abs(S.gated_errors(_t(pred2), _t(ent), _t(mc), _t(ref), _t(n), 0.5)
               ["served_max_err"] - 0.01) < 1e-12


def test_strict_fallback_size_follows_the_largest_binomial_variance():
    """A strict fallback answer's standard error stays 6 times inside the
    0.02 bound: sims = max p(1-p) * (6 / 0.02)^2, whole generations of 64,
    clamped to [1024, 2^20]."""
    from paper_2108_02419_amd import query_loop as Q
    assert Q.strict_sims(np.array([0.5, 0.5])) == 22528          # 22500 -> 352 * 64
    assert Q.strict_sims(np.array([0.9, 0.05, 0.05])) == 8128     # 0.09 * 90000 = 8100
    assert Q.strict_sims(np.array([1.0, 0.0])) == 1024            # decided race: the floor
    for p in (np.array([0.3, 0.7]), np.array([0.62, 0.2, 0.18])):
        n = Q.strict_sims(p)
        assert n % 64 == 0
        se = np.sqrt(np.max(p * (1 - p)) / n)
        assert 6 * se <= 0.02 < 6 * np.sqrt(np.max(p * (1 - p)) / (n - 64))
