"""Host-side checks of the Python binding's argument marshalling (no GPU):
the vectorised request table packs exactly what the per-request path packs."""
import ctypes

import numpy as np
import pytest

from paper_2108_02419_amd import _bbe, inputs


@pytest.fixture(scope="module")
def L():
    try:
        return _bbe.lib()
    except _bbe.BBEError as e:  # pragma: no cover - the build step makes the library
        pytest.skip(str(e))


def _floats(addr, n):
    return np.ctypeslib.as_array((ctypes.c_float * n).from_address(int(addr))).copy()


def test_request_table_matches_per_request_marshalling(L):
    specs = inputs.batch_requests(n_requests=9)
    races = [_bbe.Race(s.comp, inputs.TRACK_LEN) for s in specs]
    rng = np.random.default_rng(7)
    B = len(specs)
    tick = rng.integers(1, 500, B).astype(np.uint32)
    pos = rng.uniform(0, 1500, (B, 20)).astype(np.float32)
    prev = rng.uniform(1, 9, (B, 20)).astype(np.float32)
    sim_begin = rng.integers(0, 1000, B)
    n_sims = rng.integers(1, 5000, B)
    req = rng.integers(0, 2**32, B)
    stop = np.array([rng.integers(0, s.n + 1) for s in specs])
    listed = [(r, (int(tick[i]), pos[i, :s.n], prev[i, :s.n]), int(sim_begin[i]), int(n_sims[i]),
               int(req[i]), int(stop[i])) for i, (r, s) in enumerate(zip(races, specs))]
    arr, keep = _bbe._request_array(listed)
    tab = _bbe.RequestTable(races, n_sims, req, stop, sim_begin, tick=tick, pos=pos, prev=prev)
    packed = (_bbe.Request * B).from_address(tab.ptr)
    for i, s in enumerate(specs):
        a, b = arr[i], packed[i]
        assert a.race == b.race == races[i].handle.value
        assert (a.sim_begin, a.n_sims, a.request, a.stop_after) == \
            (b.sim_begin, b.n_sims, b.request, b.stop_after)
        sa, sb = a.state.contents, b.state.contents
        assert sa.tick == sb.tick == tick[i]
        np.testing.assert_array_equal(_floats(sb.pos, s.n), pos[i, :s.n])
        np.testing.assert_array_equal(_floats(sb.prev_step, s.n), prev[i, :s.n])
        np.testing.assert_array_equal(_floats(sa.pos, s.n), _floats(sb.pos, s.n))
    del keep


def test_request_table_start_state_and_shape_checks(L):
    specs = inputs.batch_requests(n_requests=3)
    races = [_bbe.Race(s.comp, inputs.TRACK_LEN) for s in specs]
    tab = _bbe.RequestTable(races, 100, [1, 2, 3])
    packed = (_bbe.Request * 3).from_address(tab.ptr)
    assert all(not bool(packed[i].state) for i in range(3))  # NULL: start of race
    assert [packed[i].request for i in range(3)] == [1, 2, 3]
    with pytest.raises(_bbe.BBEError):
        _bbe.RequestTable(races, 100, [1, 2, 3], tick=[1, 1, 1], pos=np.zeros((3, 2), np.float32),
                          prev=np.ones((3, 2), np.float32))


def test_race_from_rows_matches_struct_marshalling(L):
    comp = inputs.batch_requests(n_requests=1)[0].comp
    r = _bbe.Race(comp, inputs.TRACK_LEN)
    assert L.bbe_race_n(r.handle) == comp.shape[0]
    # a rejected row is reported with its index, as with struct-by-struct marshalling
    bad = comp.copy()
    bad[2, 0] = -1.0
    with pytest.raises(_bbe.BBEError) as ei:
        _bbe.Race(bad, inputs.TRACK_LEN)
    assert "competitor 2" in str(ei.value)
