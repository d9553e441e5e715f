"""End to end on the GPU: Monte-Carlo labels from the batched path, encoding,
training with the project's kernels, and what the trained network gains --
against its untrained self and against bettors with few dry-runs (RP(d),
paper Section 3), all judged by high-sample Monte-Carlo on held-out in-play
states."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from paper_2108_02419_amd import _bbe, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def test_trained_surrogate_gains(torch):
    from paper_2108_02419_amd import surrogate as S
    announce("surrogate: 30000 states x 500 sims, 80 epochs")
    specs = inputs.surrogate_states(30_000)
    rng = np.random.default_rng(0)
    specs = [specs[i] for i in rng.permutation(len(specs))]
    ds = S.gen_states(specs, 4)
    probs, _ = S.mc_probs(ds, 500, 4, request_base=0)
    x, n, _, target = S.encode(ds, probs)
    init = inputs.surrogate_init(4)
    net = _bbe.Mlp(init, max_batch=512)
    hist = S.train(net, x, n, target, epochs=80, batch=512, lr_max=2e-3)
    print(f"loss first/last epoch {hist[0]:.4f} {hist[-1]:.4f}", flush=True)
    assert hist[-1] < hist[0]

    eds = S.gen_states(inputs.surrogate_states(150, first=10_000_000), 5)
    jprobs, _ = S.mc_probs(eds, 200_000, 5, request_base=1 << 24)
    ex, en, _, jt = S.encode(eds, jprobs)
    pred, _ = S.predict(net, ex, en)
    pred0, _ = S.predict(_bbe.Mlp(init, max_batch=8), ex, en)
    e_tr, e_un = S.errors(pred, jt, en), S.errors(pred0, jt, en)
    rp = {}
    for d in [4, 16, 64]:
        few, _ = S.mc_probs(eds, d, 6 + d, request_base=(1 << 25) + d)
        _, _, _, ft = S.encode(eds, few)
        rp[d] = S.errors(ft, jt, en)
    torch.cuda.synchronize()
    print(f"trained {e_tr}\nuntrained {e_un}", flush=True)
    for d, e in rp.items():
        print(f"RP({d}) {e}", flush=True)
    assert e_tr["tv_mean"] < 0.5 * e_un["tv_mean"]
    assert e_tr["tv_mean"] < rp[4]["tv_mean"]
