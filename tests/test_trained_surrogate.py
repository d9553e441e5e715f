"""The trained surrogates shipped with the package
(paper_2108_02419_amd/trained/: one trained on races of 1-second ticks, one
on races of 0.1-second ticks): each file is what its recipe says (format,
parameter count, hash), and, evaluated by the float64 reference network on
in-play states encoded by the reference encoder, each predicts the oracle's
Monte-Carlo win probabilities far better than the untrained network does
(no GPU)."""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import mlp
from paper_2108_02419_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAINED = os.path.join(ROOT, "paper_2108_02419_amd", "trained")


NETS = {1.0: "surrogate", 0.1: "surrogate_dt01"}


def _load(dt=1.0):
    raw = open(os.path.join(TRAINED, NETS[dt] + ".bbemlp"), "rb").read()
    meta = json.load(open(os.path.join(TRAINED, NETS[dt] + ".json")))
    return raw, meta


@pytest.mark.parametrize("dt", [1.0, 0.1])
def test_file_format_and_recipe(dt):
    raw, meta = _load(dt)
    assert raw[:8] == b"BBEMLP01"
    assert int(np.frombuffer(raw[8:12], "<u4")[0]) == mlp.N_PARAMS
    assert len(raw) == 12 + 4 * mlp.N_PARAMS
    assert hashlib.sha256(raw).hexdigest() == meta["sha256"]
    p = np.frombuffer(raw[12:], "<f4")
    assert np.isfinite(p).all()
    assert meta["train_states"] >= 10_000_000 and meta["label_sims"] == 10_000
    assert meta.get("dt", 1.0) == dt


@pytest.mark.parametrize("dt", [1.0, 0.1])
def test_trained_network_predicts_the_oracle(orc, dt):
    raw, meta = _load(dt)
    params = np.frombuffer(raw[12:], "<f4").astype(np.float64)
    # states no training block drew
    a = inputs.surrogate_state_block(9999, 24, dict(inputs.CFG_SURROGATE, dt=dt))
    L = inputs.TRACK_LEN
    err_t, err_u = [], []
    init = inputs.surrogate_init(4).astype(np.float64)
    for i in range(24):
        k = int(a["n"][i])
        comp = a["comp"][i, :k]
        st = orc.race_prefix(comp, L, 4, int(a["prefix_request"][i]), 0, float(a["target"][i]))
        _, w, _ = orc.race_sim(comp, L, 4000, 11, request=i, state=st, stop_after=1,
                               want_orders=False, threads=8)
        p_mc = orc.win_probs(w)
        cb = np.zeros((1, 20, 5), np.float32)
        cb[0, :k] = comp
        pos = np.zeros((1, 20), np.float32)
        prev = np.zeros((1, 20), np.float32)
        pos[0, :k], prev[0, :k] = st[1], st[2]
        X, slot = mlp.encode(cb, [k], pos, prev, L, dt)
        for net, out in ((params, err_t), (init, err_u)):
            _, q, _ = mlp.forward(net, mlp.bf16(X), [k])
            pc = np.zeros(k)
            for r in range(k):
                pc[slot[0, r]] = q[0, r]
            out.append(0.5 * np.abs(pc - p_mc).sum())
    # total variation against 4000-simulation Monte-Carlo (its own noise is
    # about 0.01-0.03 per state)
    print(f"dt {dt}: total variation, trained {np.mean(err_t):.4f}, untrained {np.mean(err_u):.4f}")
    assert np.mean(err_t) < 0.06, np.mean(err_t)
    assert np.mean(err_t) < 0.4 * np.mean(err_u), (np.mean(err_t), np.mean(err_u))
