"""The allocation-free form of the in-play state batch
(bbe_prefix_batch_noalloc) through the C ABI: the same outputs as
bbe_prefix_batch on two calls in a row, the second with fewer requests
(the fixed workspace keeps the first call's descriptors past the second's
end), bit for bit; both also equal the oracle's states."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from paper_2108_02419_amd import _bbe, inputs
from paper_2108_02419_amd._bbe import Race

pytestmark = pytest.mark.gpu
L = inputs.TRACK_LEN
SEED = 11


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _run(torch, fn, tab, sims, targets):
    B = len(tab)
    tick = torch.full((B,), -7, dtype=torch.int32, device="cuda")
    pos = torch.full((B, 20), -1.0, dtype=torch.float32, device="cuda")
    prev = torch.full((B, 20), -1.0, dtype=torch.float32, device="cuda")
    fn(tab, sims, targets, SEED, tick, pos, prev)
    torch.cuda.synchronize()
    return tick.cpu().numpy().view(np.uint32), pos.cpu().numpy(), prev.cpu().numpy()


def test_noalloc_prefix_batch_matches_allocating_form(torch, orc):
    reqs = inputs.batch_requests(n_requests=700)
    races = [Race(r.comp, L) for r in reqs]
    rng = np.random.default_rng(2)
    for B in (700, 133):  # the second call smaller than the first
        sub = reqs[:B]
        tab = _bbe.RequestTable(races[:B], 1, [r.prefix_request for r in sub])
        sims = rng.integers(0, 1000, B).astype(np.uint32)
        targets = np.array([r.target for r in sub], np.float32)
        targets[::5] = np.float32(L - 1e-3)  # some races reach the line first
        announce(f"prefix batch noalloc B={B}")
        want = _run(torch, _bbe.prefix_batch, tab, sims, targets)
        got = _run(torch, _bbe.prefix_batch_noalloc, tab, sims, targets)
        for w, g in zip(want, got):
            np.testing.assert_array_equal(g, w)
        assert (got[0] == 0xFFFFFFFF).any() and (got[0] != 0xFFFFFFFF).any()
        for i in rng.choice(B, 12, replace=False):
            r = sub[i]
            if got[0][i] == 0xFFFFFFFF:
                continue
            t, p, q = orc.race_prefix(r.comp, L, SEED, r.prefix_request, int(sims[i]),
                                      targets[i])
            assert got[0][i] == t
            np.testing.assert_array_equal(got[1][i, :r.n], p)
            np.testing.assert_array_equal(got[2][i, :r.n], q)

