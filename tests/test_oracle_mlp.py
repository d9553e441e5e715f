"""Pins of the float64 surrogate reference (oracle/mlp.py): central finite
differences of the loss, closed forms of softmax cross-entropy and of the
first Adam step, and properties of the state encoding."""
import numpy as np

from oracle import mlp


def _rand_net(rng, scale=0.2):
    return rng.normal(0, scale, size=mlp.N_PARAMS)


def _batch(rng, B):
    X = rng.normal(0, 1, size=(B, mlp.IN))
    n = rng.integers(1, 21, size=B)
    n[0] = 20
    T = rng.random((B, mlp.OUT)) * (np.arange(mlp.OUT)[None, :] < n[:, None])
    T /= T.sum(axis=1, keepdims=True)
    return X, n, T


def test_parameter_count():
    assert mlp.N_PARAMS == 177_940


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _rand_net(rng)
    X, n, T = _batch(rng, 6)
    loss, g = mlp.loss_and_grad(p, X, n, T, bf16_on=False)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 150, replace=False),
                          np.arange(mlp.N_PARAMS - 20, mlp.N_PARAMS),   # b4
                          np.arange(160 * 256, 160 * 256 + 10)])        # b1
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, X, n, T, bf16_on=False)
        lm, _ = mlp.loss_and_grad(p - e, X, n, T, bf16_on=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_softmax_cross_entropy_closed_forms():
    rng = np.random.default_rng(1)
    p = _rand_net(rng)
    X, n, T = _batch(rng, 5)
    z, q, _ = mlp.forward(p, X, n, bf16_on=False)
    # probabilities on the valid slots only, summing to one
    for b in range(5):
        assert (q[b, n[b]:] == 0).all()
        assert abs(q[b, :n[b]].sum() - 1) < 1e-12
    # shifting b4 (every logit by the same constant) changes nothing
    P = mlp.unpack(p)
    P["b4"] = P["b4"] + 3.25
    _, q2, _ = mlp.forward(mlp.pack(P), X, n, bf16_on=False)
    np.testing.assert_allclose(q2, q, atol=1e-12)
    # loss against the network's own output is its entropy (mean)
    loss, g = mlp.loss_and_grad(p, X, n, q, bf16_on=False)
    assert abs(loss - mlp.entropy(q).mean()) < 1e-12
    # ... and its gradient vanishes
    assert np.abs(g).max() < 1e-12


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 1.0 + 2**-9, -2.5, 0.0, 3.0e38])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0          # halfway, ties to even (mantissa 0)
    assert r[2] == 1.0 + 2**-7  # 1.5 ulps rounds up
    assert r[3] == 1.0          # below halfway
    assert r[4] == -2.5 and r[5] == 0.0
    assert mlp.bf16(1.0 + 3 * 2**-8) == 1.0 + 2**-6  # halfway, ties to even (mantissa 2)


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    lr = 1e-3
    w1, m, v = mlp.adam(w, g, np.zeros(50), np.zeros(50), 1, lr)
    # bias-corrected first moments equal g and g^2, so the step is lr*g/(|g|+eps)
    np.testing.assert_allclose(w1, w - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_encoding_by_hand_and_label_invariance():
    comp = np.zeros((1, 20, 5), np.float32)
    comp[0, :3] = [[5, 9, 1, 0.1, 2], [6, 8, 1, -0.2, 1], [4, 10, 1, 0, 3]]
    pos = np.zeros((1, 20), np.float32)
    prev = np.zeros((1, 20), np.float32)
    pos[0, :3] = [1000, 1500, 1000]
    prev[0, :3] = [0.75, 0.6, 0.5]
    X, slot = mlp.encode(comp, [3], pos, prev, 2000.0, 0.1)
    assert slot[0, :4].tolist() == [1, 0, 2, -1]  # smallest expected remaining ticks first
    f = X.reshape(20, 8)
    # worked by hand (dt = 0.1: step scale 0.75, leader-gap scale 7.5, speed scale 1.5);
    # remaining ticks T = (L-d) / (mean step * (1 + rho*d/L)):
    #   c0: 1000 / (7 * 1.05) = 136.0544218, c1: 500 / (7 * 0.85) = 84.0336134,
    #   c2: 1000 / 7 = 142.8571429; best T is c1's
    want = np.array([
        # rem   lead       gap  s/v     spd     noise   rho/.2 (T - Tmin)/10
        [0.25, 0.0,       4.0, 0.8,    9.33333, 1 / 7., -1.0, 0.0],        # c1, leader
        [0.5,  66.666667, 4.0, 1.0,    9.33333, 2 / 7., 0.5,  5.2020808],  # c0 (gap 666 -> 4)
        [0.5,  66.666667, 0.0, 0.666667, 9.33333, 3 / 7., 0.0, 5.8823529],  # c2, tied with c0
    ])
    np.testing.assert_allclose(f[:3], want, rtol=2e-6, atol=1e-7)
    assert (f[3:] == 0).all()
    # slots follow the expected remaining ticks, not the track: a faster
    # competitor just behind takes slot 0; its gap is to the one ahead on
    # the track, whose own gap is the leader's 4
    c2 = np.zeros((1, 20, 5), np.float32)
    c2[0, :2] = [[4, 6, 1, 0, 2], [8, 10, 1, 0, 2]]
    p2 = np.zeros((1, 20), np.float32)
    p2[0, :2] = [1000, 999]
    s2 = np.zeros((1, 20), np.float32)
    s2[0, :2] = [0.5, 0.9]
    X2, sl2 = mlp.encode(c2, [2], p2, s2, 2000.0, 0.1)
    assert sl2[0, :3].tolist() == [1, 0, -1]
    # T: c1 1001 / 9 = 111.2222, c0 1000 / 5 = 200
    want2 = np.array([
        [0.5005, 1 / 7.5, 1 / 0.75, 1.2,      12.0,    1 / 9., 0.0, 0.0],
        [0.5,    0.0,     4.0,      0.666667, 6.666667, 0.2,   0.0, 8.8777778],
    ])
    np.testing.assert_allclose(X2.reshape(20, 8)[:2], want2, rtol=2e-6, atol=1e-6)
    # relabelling the competitors changes nothing in the encoding (no ties:
    # tied competitors are ordered by index, and the gap feature follows it)
    pos[0, 2] = 900.0
    X, slot = mlp.encode(comp, [3], pos, prev, 2000.0, 0.1)
    perm = [2, 0, 1]
    comp2 = comp.copy()
    pos2, prev2 = pos.copy(), prev.copy()
    comp2[0, :3] = comp[0, perm]
    pos2[0, :3] = pos[0, perm]
    prev2[0, :3] = prev[0, perm]
    X2, slot2 = mlp.encode(comp2, [3], pos2, prev2, 2000.0, 0.1)
    np.testing.assert_array_equal(X, X2)
    assert [perm[c] for c in slot2[0, :3]] == slot[0, :3].tolist()


def test_accumulation_bound_holds_for_float32_sums_in_any_order():
    """The per-element bound used by the layer checks: float32 sums of
    bfloat16 products, taken in four different orders (sequential both
    ways, pairwise, shuffled), stay within accumulation_bound of the exact
    sum; the bound is a small multiple of the worst observed error."""
    rng = np.random.default_rng(11)
    worst_ratio = 0.0
    for K in (32, 160, 256):
        h = mlp.bf16(np.maximum(rng.normal(0, 1, size=(40, K)), 0))
        W = rng.uniform(-0.2, 0.2, size=(24, K))
        b = rng.uniform(-0.5, 0.5, size=24)
        a, e = mlp.dense_with_bound(h, W, b)
        Wb = mlp.bf16(W).astype(np.float32)
        hf = h.astype(np.float32)
        for r in range(h.shape[0]):
            for n in range(W.shape[0]):
                terms = list((hf[r] * Wb[n]).astype(np.float32)) + [np.float32(b[n])]
                orders = [terms, terms[::-1], [terms[i] for i in rng.permutation(len(terms))]]
                sums = []
                for t in orders:
                    acc = np.float32(0)
                    for x in t:
                        acc = np.float32(acc + x)
                    sums.append(acc)
                pair = np.asarray(terms, np.float32)
                while pair.size > 1:
                    if pair.size % 2:
                        pair = np.append(pair, np.float32(0))
                    pair = (pair[0::2] + pair[1::2]).astype(np.float32)
                sums.append(pair[0])
                for s in sums:
                    err = abs(float(s) - a[r, n])
                    assert err <= e[r, n], (K, r, n, err, e[r, n])
                    worst_ratio = max(worst_ratio, err / e[r, n])
    assert worst_ratio < 0.5


def test_bf16_interval_brackets_rounding_and_catches_a_dropped_bias():
    """Every float32 in [a - e, a + e] rounds (after ReLU) into the
    interval; the interval is a single value away from rounding
    boundaries; leaving out a bias moves the value outside it."""
    rng = np.random.default_rng(12)
    h = mlp.bf16(np.maximum(rng.normal(0, 1, size=(64, 256)), 0))
    W = rng.uniform(-0.06, 0.06, size=(256, 256))
    b = rng.uniform(-0.5, 0.5, size=256)
    a, e = mlp.dense_with_bound(h, W, b)
    lo, hi = mlp.bf16_interval(a, e, relu=True)
    for frac in (-1.0, -0.5, 0.0, 0.5, 1.0):
        v = mlp.bf16(np.maximum(a + frac * e, 0.0))
        assert ((v >= lo) & (v <= hi)).all()
    assert (lo == hi).mean() > 0.8
    a_nobias, _ = mlp.dense_with_bound(h, W)
    v = mlp.bf16(np.maximum(a_nobias, 0.0))
    outside = (v < lo) | (v > hi)
    assert outside.mean() > 0.5
