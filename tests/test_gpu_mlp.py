"""GPU parity of the surrogate kernels against the float64 reference
(oracle/mlp.py) on the same seeded inputs: the encoder bit for bit, the
forward pass and the gradients within tolerances derived from bfloat16
operands with float32 accumulation, Adam within 1e-6 relative."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from oracle import mlp as ref
from paper_2108_02419_amd import _bbe, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _features(rng, B):
    """Random bfloat16-exact feature rows, valid-slot counts and targets."""
    X = ref.bf16(rng.normal(0, 1, size=(B, ref.IN)))
    n = rng.integers(1, 21, size=B).astype(np.int32)
    n[: min(B, 3)] = [20, 1, 7][: min(B, 3)]
    T = rng.random((B, ref.OUT)) * (np.arange(ref.OUT)[None, :] < n[:, None])
    T /= T.sum(axis=1, keepdims=True)
    return X, n, T.astype(np.float32)


def _bits(torch, X):
    u = np.asarray(X, np.float32).view(np.uint32) >> 16
    return torch.tensor(u.astype(np.uint16).view(np.int16), device="cuda")


def _bf16_of_bits(h):
    """bfloat16 bit patterns (int16 CUDA tensor) -> float64 numpy."""
    u = h.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _check_layers(torch, net, params, X, n):
    """Each layer of the GPU forward pass checked on its own GPU inputs:
    h_k must be one of the bfloat16 values that rounding ReLU(h_{k-1} W_k^T +
    b_k), evaluated with float32 accumulation in any order, can give
    (oracle/mlp.py accumulation_bound: Higham's gamma_m for m products and
    the bias); the logits must lie within that bound of h3 W4^T + b4.  A
    dropped bias or a wrong operand moves most elements outside.  Returns
    the GPU logits [B, 20] and the GPU probabilities."""
    B = X.shape[0]
    xt, nt = _bits(torch, X), torch.tensor(n, device="cuda")
    hidden = torch.empty((3, B, 256), dtype=torch.int16, device="cuda")
    logits = torch.empty((B, 32), dtype=torch.float32, device="cuda")
    logits2 = torch.empty((B, 32), dtype=torch.float32, device="cuda")
    probs = torch.empty((B, 20), dtype=torch.float32, device="cuda")
    ent = torch.empty(B, dtype=torch.float32, device="cuda")
    net.forward_hidden(xt, nt, hidden, logits)
    net.forward(xt, nt, probs, ent, logits2)
    torch.cuda.synchronize()
    H = _bf16_of_bits(hidden)
    P = ref.unpack(np.asarray(params, np.float32).astype(np.float64))
    inp = ref.bf16(X)
    for k in range(3):
        a, e = ref.dense_with_bound(inp, P[f"W{k + 1}"], P[f"b{k + 1}"])
        lo, hi = ref.bf16_interval(a, e, relu=True)
        bad = (H[k] < lo) | (H[k] > hi)
        assert not bad.any(), (k + 1, int(bad.sum()), np.argwhere(bad)[:4].tolist())
        inp = H[k]
    z, e = ref.dense_with_bound(inp, P["W4"], P["b4"])
    zg = logits.cpu().numpy().astype(np.float64)[:, :20]
    mask = np.arange(20)[None, :] < n[:, None]
    assert (np.abs(zg - z) <= e)[mask].all(), np.abs(zg - z)[mask].max()
    assert np.isneginf(zg[~mask]).all()
    np.testing.assert_array_equal(logits2.cpu().numpy()[:, :20], logits.cpu().numpy()[:, :20])
    # softmax and entropy of the GPU's own logits (float32 exp/log on the GPU)
    zm = np.where(mask, zg, -np.inf)
    ex = np.where(mask, np.exp(zm - zm.max(axis=1, keepdims=True)), 0.0)
    q = ex / ex.sum(axis=1, keepdims=True)
    np.testing.assert_allclose(probs.cpu().numpy(), q, rtol=0, atol=5e-6)
    np.testing.assert_allclose(ent.cpu().numpy(), ref.entropy(q), rtol=0, atol=2e-5)
    return zg, probs.cpu().numpy()


def test_forward_layer_by_layer_with_biases(torch):
    """Random non-zero biases, batches of one tile, ragged tails and several
    tiles; also checked end to end against the reference from the features
    alone (within 2e-3 on the probabilities)."""
    rng = np.random.default_rng(0)
    params = inputs.surrogate_random(4)
    for B in [1, 63, 64, 200]:  # one tile, ragged tails, several tiles
        announce(f"mlp forward per layer B={B}")
        X, n, _ = _features(rng, B)
        net = _bbe.Mlp(params, max_batch=256)
        _, pg = _check_layers(torch, net, params, X, n)
        _, q, _ = ref.forward(params.astype(np.float64), X, n)
        np.testing.assert_allclose(pg, q, atol=2e-3)


def _check_rows(H, zg, params, X, n, sel):
    """The per-layer check of _check_layers on rows `sel` of a batch whose
    hidden activations H [3, B, 256] and logits zg [B, 20] the GPU returned."""
    P = ref.unpack(np.asarray(params, np.float32).astype(np.float64))
    inp = ref.bf16(X[sel])
    for k in range(3):
        a, e = ref.dense_with_bound(inp, P[f"W{k + 1}"], P[f"b{k + 1}"])
        lo, hi = ref.bf16_interval(a, e, relu=True)
        h = H[k][sel]
        assert not ((h < lo) | (h > hi)).any(), k + 1
        inp = h
    z, e = ref.dense_with_bound(inp, P["W4"], P["b4"])
    mask = np.arange(20)[None, :] < n[sel][:, None]
    assert (np.abs(zg[sel] - z) <= e)[mask].all()


def test_row_tiles_of_every_size_give_the_same_rows(torch):
    """Batches large enough for 32- and 64-row workgroups (8200 and 16400
    rows, both ragged) pass the per-layer check on their first and last
    rows, and a row's logits are the same bits whichever tile size its
    batch gets (16 rows at 200)."""
    rng = np.random.default_rng(9)
    params = inputs.surrogate_random(3)
    net = _bbe.Mlp(params, max_batch=8)
    X, n, _ = _features(rng, 16400)
    outs = {}
    for B in (200, 8200, 16400):
        announce(f"mlp forward row tiles B={B}")
        xt, nt = _bits(torch, X[:B]), torch.tensor(n[:B], device="cuda")
        hidden = torch.empty((3, B, 256), dtype=torch.int16, device="cuda")
        logits = torch.empty((B, 32), dtype=torch.float32, device="cuda")
        net.forward_hidden(xt, nt, hidden, logits)
        torch.cuda.synchronize()
        zg = logits.cpu().numpy()[:, :20].astype(np.float64)
        outs[B] = zg
        sel = np.r_[0:min(B, 300), max(0, B - 300):B]  # the first tiles and the ragged tail
        _check_rows(_bf16_of_bits(hidden), zg, params, X[:B], n[:B], sel)
    np.testing.assert_array_equal(outs[8200][:200], outs[200])
    np.testing.assert_array_equal(outs[16400][:8200], outs[8200])


def test_gradients_with_large_row_tiles(torch):
    """The backward-data kernel at 64-row tiles (16400 rows) against the
    reference."""
    rng = np.random.default_rng(10)
    params = inputs.surrogate_random(2)
    X, n, T = _features(rng, 16400)
    net = _bbe.Mlp(params, max_batch=16400)
    announce("mlp gradients B=16400")
    _grad_check(torch, net, params, X, n, T)


def test_forward_layer_by_layer_after_adam_steps(torch):
    """After training steps the kernels use the refreshed bfloat16 copies of
    the updated master parameters, biases included."""
    rng = np.random.default_rng(6)
    params = inputs.surrogate_random(5)
    X, n, T = _features(rng, 256)
    net = _bbe.Mlp(params, max_batch=256)
    xt, nt, tt = _bits(torch, X), torch.tensor(n, device="cuda"), torch.tensor(T, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    announce("mlp 5 Adam steps, then forward per layer")
    for _ in range(5):
        net.train_step(xt, nt, tt, 3e-3, loss)
    torch.cuda.synchronize()
    trained = net.params()
    moved = ref.unpack(trained.astype(np.float64))
    start = ref.unpack(params.astype(np.float64))
    for name in moved:  # every tensor, biases too, was updated
        assert not np.array_equal(moved[name], start[name]), name
    Xe, ne, _ = _features(rng, 130)
    _check_layers(torch, net, trained, Xe, ne)


def _grad_check(torch, net, params, X, n, T):
    B = X.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    grad = torch.empty(_bbe.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    net.loss_grad(_bits(torch, X), torch.tensor(n, device="cuda"),
                  torch.tensor(T, device="cuda"), loss, grad)
    torch.cuda.synchronize()
    l_ref, g_ref = ref.loss_and_grad(np.asarray(params, np.float32).astype(np.float64), X, n, T)
    assert abs(loss.item() - l_ref) <= 1e-4 * abs(l_ref), (B, loss.item(), l_ref)
    g = grad.cpu().numpy().astype(np.float64)
    G, R = ref.unpack(g), ref.unpack(g_ref)
    for name in G:
        err = np.linalg.norm(G[name] - R[name]) / max(np.linalg.norm(R[name]), 1e-30)
        assert err <= 1e-3, (name, err)
    return grad.cpu().numpy()


def test_gradients_match_reference(torch):
    """Non-zero biases; the bias gradients are compared like the weights'."""
    rng = np.random.default_rng(1)
    params = inputs.surrogate_random(4)
    X, n, T = _features(rng, 300)
    net = _bbe.Mlp(params, max_batch=512)
    announce("mlp gradients B=300 with biases")
    _grad_check(torch, net, params, X, n, T)


def test_gradients_match_reference_after_adam_steps(torch):
    rng = np.random.default_rng(7)
    params = inputs.surrogate_random(6)
    X, n, T = _features(rng, 200)
    net = _bbe.Mlp(params, max_batch=256)
    xt, nt, tt = _bits(torch, X), torch.tensor(n, device="cuda"), torch.tensor(T, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    announce("mlp 4 Adam steps, then gradients")
    for _ in range(4):
        net.train_step(xt, nt, tt, 3e-3, loss)
    torch.cuda.synchronize()
    X2, n2, T2 = _features(rng, 200)
    _grad_check(torch, net, net.params(), X2, n2, T2)


def test_gradients_are_reproducible_over_several_row_chunks(torch):
    """1000 rows (four 256-row chunks of the weight-gradient kernel): the
    gradient matches the reference and two calls give the same bits."""
    rng = np.random.default_rng(5)
    params = inputs.surrogate_random(4)
    B = 1000
    X, n, T = _features(rng, B)
    announce(f"mlp gradients B={B}, twice")
    net = _bbe.Mlp(params, max_batch=1024)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    grads = []
    for _ in range(2):
        grad = torch.empty(_bbe.MLP_NPARAMS, dtype=torch.float32, device="cuda")
        net.loss_grad(_bits(torch, X), torch.tensor(n, device="cuda"),
                      torch.tensor(T, device="cuda"), loss, grad)
        torch.cuda.synchronize()
        grads.append(grad.cpu().numpy())
    np.testing.assert_array_equal(grads[0], grads[1])
    _, g_ref = ref.loss_and_grad(params.astype(np.float64), X, n, T)
    G, R = ref.unpack(grads[0].astype(np.float64)), ref.unpack(g_ref)
    for name in G:
        err = np.linalg.norm(G[name] - R[name]) / max(np.linalg.norm(R[name]), 1e-30)
        assert err <= 1e-3, (name, err)


def test_adam_matches_reference(torch):
    rng = np.random.default_rng(2)
    params = inputs.surrogate_init(4)
    net = _bbe.Mlp(params, max_batch=8)
    p = params.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4):
        g = rng.normal(0, 1e-3, size=p.shape)
        p, m, v = ref.adam(p, g, m, v, step, 1e-3)
        net.adam_step(1e-3, grad=torch.tensor(g.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    got = net.params().astype(np.float64)
    np.testing.assert_allclose(got, p, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("B", [64, 37])
def test_encoder_bit_exact(torch, B):
    """Two states per wave: an even batch and a ragged one (the last wave's
    second half holds no state); exact position ties, two identical
    competitors side by side (equal expected times) and a one-competitor
    state exercise the slot order and the gap feature."""
    reqs = inputs.surrogate_states(B)
    reqs[7] = inputs.RequestSpec(index=7, comp=reqs[7].comp[:1], remaining=reqs[7].remaining,
                                 target=reqs[7].target, n_sims=reqs[7].n_sims,
                                 prefix_request=reqs[7].prefix_request)
    import oracle
    comp = np.zeros((B, 20, 5), np.float32)
    pos = np.zeros((B, 20), np.float32)
    prev = np.zeros((B, 20), np.float32)
    n = np.array([r.n for r in reqs], np.int32)
    for i, r in enumerate(reqs):
        comp[i, :r.n] = r.comp
        t, p, q = oracle.race_prefix(r.comp, inputs.TRACK_LEN, 4, r.prefix_request, 0, r.target)
        pos[i, :r.n], prev[i, :r.n] = p, q
    pos[5, :3] = pos[5, 3]  # exact ties exercise the slot order
    if reqs[9].n >= 2:  # two identical competitors side by side: equal T, index order
        comp[9, 1], pos[9, 1], prev[9, 1] = comp[9, 0], pos[9, 0], prev[9, 0]
    X, slot = ref.encode(comp, n, pos, prev, inputs.TRACK_LEN, 0.1)
    x = torch.full((B, 160), 77, dtype=torch.int16, device="cuda")
    s = torch.full((B, 20), 77, dtype=torch.int32, device="cuda")
    probs = np.random.default_rng(B).random((B, 20))
    tgt = torch.full((B, 20), 7.0, dtype=torch.float32, device="cuda")
    _bbe.encode_states(torch.tensor(comp, device="cuda"), torch.tensor(n, device="cuda"),
                       torch.tensor(pos, device="cuda"), torch.tensor(prev, device="cuda"),
                       inputs.TRACK_LEN, 0.1, x, s, torch.tensor(probs, device="cuda"), tgt)
    torch.cuda.synchronize()
    want = (ref.bf16(X).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    np.testing.assert_array_equal(x.cpu().numpy().view(np.uint16), want)
    np.testing.assert_array_equal(s.cpu().numpy(), slot)
    # labels follow the slots: target[b][r] = probs[b][competitor in slot r], 0 in padding
    want_t = np.where(slot >= 0, np.take_along_axis(probs, np.maximum(slot, 0), axis=1), 0.0)
    np.testing.assert_array_equal(tgt.cpu().numpy(), want_t.astype(np.float32))


def test_training_reduces_loss(torch):
    rng = np.random.default_rng(3)
    params = inputs.surrogate_init(4)
    B = 512
    X, n, T = _features(rng, B)
    net = _bbe.Mlp(params, max_batch=B)
    xt, nt, tt = _bits(torch, X), torch.tensor(n, device="cuda"), torch.tensor(T, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    for _ in range(60):
        net.train_step(xt, nt, tt, 1e-3, loss)
        losses.append(loss.item())
    ent = float(np.mean([-(t[t > 0] * np.log(t[t > 0])).sum() for t in T]))
    assert losses[-1] < losses[0] - 0.5 * (losses[0] - ent), (losses[0], losses[-1], ent)


def test_save_and_load_round_trip(torch, tmp_path):
    """A network trained for a few steps, saved and loaded: identical
    parameters and identical forward outputs."""
    rng = np.random.default_rng(5)
    net = _bbe.Mlp(inputs.surrogate_init(4), max_batch=64)
    X, n, T = _features(rng, 64)
    xt, nt = _bits(torch, X), torch.tensor(n, device="cuda")
    tt = torch.tensor(T, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.train_step(xt, nt, tt, 1e-3, loss)
    torch.cuda.synchronize()
    path = str(tmp_path / "net.bin")
    announce("mlp save/load")
    net.save(path)
    back = _bbe.Mlp.load(path, max_batch=8)
    np.testing.assert_array_equal(back.params(), net.params())
    outs = []
    for m in (net, back):
        probs = torch.empty((64, 20), dtype=torch.float32, device="cuda")
        m.forward(xt, nt, probs)
        torch.cuda.synchronize()
        outs.append(probs.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


def test_checkpoint_resumes_training_exactly(torch, tmp_path):
    """Six training steps on six minibatches straight through, and three
    steps, a checkpoint, a fresh network loaded from it and the last three
    steps: the two checkpoints after six steps are the same bytes
    (parameters, both Adam moments, step count).  Loading the parameters
    alone (Adam state reset) gives a different network."""
    rng = np.random.default_rng(21)
    B = 300
    batches = []
    for _ in range(6):
        X, n, T = _features(rng, B)
        batches.append((_bits(torch, X), torch.tensor(n, device="cuda"),
                        torch.tensor(T, device="cuda")))
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    params = inputs.surrogate_random(6)
    announce("mlp checkpoint resume")

    def steps(net, bs):
        for xt, nt, tt in bs:
            net.train_step(xt, nt, tt, 2e-3, loss)
        torch.cuda.synchronize()

    a = _bbe.Mlp(params, max_batch=B)
    steps(a, batches)
    a.save_checkpoint(str(tmp_path / "a.ckpt"))

    b = _bbe.Mlp(params, max_batch=B)
    steps(b, batches[:3])
    b.save_checkpoint(str(tmp_path / "b3.ckpt"))
    b.save(str(tmp_path / "b3.params"))
    c = _bbe.Mlp.load(str(tmp_path / "b3.ckpt"), max_batch=B)
    steps(c, batches[3:])
    c.save_checkpoint(str(tmp_path / "c.ckpt"))
    raw_a = open(tmp_path / "a.ckpt", "rb").read()
    assert raw_a[:8] == b"BBEMLP02" and len(raw_a) == 8 + 4 + 8 + 3 * 4 * ref.N_PARAMS
    assert int(np.frombuffer(raw_a[12:20], "<u8")[0]) == 6
    assert raw_a == open(tmp_path / "c.ckpt", "rb").read()

    d = _bbe.Mlp.load(str(tmp_path / "b3.params"), max_batch=B)
    steps(d, batches[3:])
    assert not np.array_equal(d.params(), a.params())
