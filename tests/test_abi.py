"""The C ABI boundary without a GPU: the library loads, exports every
function include/*.h declares, and rejects invalid arguments before any
device work (so these run on the CPU)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2108_02419_amd import _bbe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(bbe_[a-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_bbe.LIB_PATH):
        pytest.skip("libbbe.so not built")
    return _bbe.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "bbe_race_sim" in names and "bbe_race_init" in names
    for name in names:
        assert hasattr(L, name), name
    assert names <= set(_bbe.SIGNATURES), names - set(_bbe.SIGNATURES)


GOOD = [[5.0, 8.0, 1.0, 0.1, 2.0]] * 3


@pytest.mark.parametrize("comp,track", [
    (GOOD[:0], 2000.0), ([[5, 8, 1, 0.1, 2]] * 21, 2000.0), ([[0, 8, 1, 0, 2]], 2000.0),
    ([[5, 4, 1, 0, 2]], 2000.0), ([[5, 8, 0, 0, 2]], 2000.0), ([[5, 8, 1.5, 0, 2]], 2000.0),
    ([[5, 8, 1, 1.0, 2]], 2000.0), ([[5, 8, 1, 0, -1]], 2000.0), ([[np.nan, 8, 1, 0, 2]], 2000.0),
    (GOOD, 0.0), (GOOD, np.inf), ([[1e-4, 8, 1, 0, 2]], 2000.0),
    # a nonzero scaled span below 2^-102
    ([[1e-32, float(np.nextafter(np.float32(1e-32), np.float32(1))), 1, 0, 2]], 1e-30),
])
def test_race_init_rejects(L, comp, track):
    """Every documented rule of bbe_race_init rejects with BBE_EINVAL."""
    with pytest.raises(_bbe.BBEError) as ei:
        _bbe.Race(np.array(comp, np.float32).reshape(-1, 5), track)
    assert ei.value.code == _bbe.EINVAL
    assert len(str(ei.value)) > 8


def test_race_sim_rejects_before_device_work(L):
    race = _bbe.Race(np.array(GOOD, np.float32), 2000.0)
    h = race.handle
    null = ctypes.c_void_p()
    cases = [
        dict(n_sims=0), dict(stop_after=0), dict(stop_after=4),
        dict(sim_begin=2**32 - 5, n_sims=10),
    ]
    for kw in cases:
        a = dict(sim_begin=0, n_sims=10, stop_after=3)
        a.update(kw)
        rc = L.bbe_race_sim(h, None, a["sim_begin"], a["n_sims"], 1, 0, a["stop_after"], null,
                            null, null, null)
        assert rc == _bbe.EINVAL, kw
        assert L.bbe_last_error().decode()
    bad_states = [
        (3, [0, 10, 2000], [1, 1, 1]), (3, [0, -1, 20], [1, 1, 1]), (3, [0, 1, 20], [1, 0, 1]),
        (3, [0, 1, np.nan], [1, 1, 1]), (2**32 - 10, [0, 0, 0], [1, 1, 1]),
    ]
    for t, p, q in bad_states:
        st, keep = _bbe._state_struct((t, np.array(p, np.float32), np.array(q, np.float32)), 3)
        rc = L.bbe_race_sim(h, ctypes.byref(st), 0, 10, 1, 0, 3, null, null, null, null)
        assert rc == _bbe.EINVAL, (t, p, q)
    assert L.bbe_race_sim(None, None, 0, 10, 1, 0, 3, null, null, null, null) == _bbe.EINVAL
    assert L.bbe_win_probs(None, 1, 3, 3, None, None) == _bbe.EINVAL
    assert L.bbe_race_prefix(h, None, 1, 0, 0, 2000.0, null, null, null, null) == _bbe.EINVAL
    buf = ctypes.c_void_p(16)  # never dereferenced: rejected before any device work
    for n in (0, 21):
        assert L.bbe_rank_counts(buf, 10, n, buf, None) == _bbe.EINVAL
    assert L.bbe_rank_counts(buf, 10, 5, None, None) == _bbe.EINVAL
    assert L.bbe_rank_counts(None, 10, 5, buf, None) == _bbe.EINVAL
    for n in (0, 8):
        assert L.bbe_order_pmf(buf, 10, n, buf, None) == _bbe.EINVAL
    assert L.bbe_order_pmf(None, 3, 4, buf, None) == _bbe.EINVAL


def test_last_error_cleared_on_success(L):
    _bbe.Race(np.array(GOOD, np.float32), 2000.0)
    assert L.bbe_last_error().decode() == ""


def test_batch_plan_rejects_before_device_work(L):
    race = _bbe.Race(np.array(GOOD, np.float32), 2000.0)
    null = ctypes.c_void_p()
    out = ctypes.c_void_p()
    fake_out = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    bad = [
        [(race, None, 0, 0, 0, 0)],                 # n_sims = 0
        [(race, None, 0, 10, 0, 4)],                # stop_after > n
        [(race, None, 2**32 - 5, 10, 0, 0)],        # range beyond 2^32
        [(race, (3, np.array([0, 1, 2001], np.float32), np.ones(3, np.float32)), 0, 10, 0, 0)],
    ]
    for specs in bad:
        arr, keep = _bbe._request_array(specs)
        rc = L.bbe_batch_plan_create(arr, len(specs), 1, fake_out, null, null, 0, null,
                                     ctypes.byref(out))
        assert rc == _bbe.EINVAL, specs
        assert L.bbe_last_error().decode()
    arr, keep = _bbe._request_array([(race, None, 0, 10, 0, 0)])
    assert L.bbe_batch_plan_create(arr, 0, 1, fake_out, null, null, 0, null,
                                   ctypes.byref(out)) == _bbe.EINVAL
    assert L.bbe_batch_plan_create(arr, 1, 1, null, null, null, 0, null,
                                   ctypes.byref(out)) == _bbe.EINVAL
    assert L.bbe_batch_plan_launch(None, None) == _bbe.EINVAL
    rc = L.bbe_prefix_batch(arr, np.zeros(1, np.uint32).ctypes.data,
                            np.array([5000.0], np.float32).ctypes.data, 1, 1, fake_out,
                            fake_out, fake_out, null)
    assert rc == _bbe.EINVAL  # target beyond the track


def test_bettors_reject_before_device_work(L):
    out = ctypes.c_void_p()
    bad = [
        ([4], [0.0]),                      # unknown kind
        ([3], [0.0]), ([3], [1.5]), ([3], [2.0 ** 21]), ([3], [np.nan]),  # LinEx window
        ([2], [-1.0]), ([2], [np.inf]), ([2], [np.nan]),                  # UD distance
        ([0, 1, 9], [0.0, 0.0, 0.0]),
    ]
    for kinds, params in bad:
        k = np.array(kinds, np.uint8)
        p = np.array(params, np.float32)
        rc = L.bbe_bettors_create(k.ctypes.data, p.ctypes.data, len(kinds), ctypes.byref(out))
        assert rc == _bbe.EINVAL, (kinds, params)
        assert L.bbe_last_error().decode()
    k = np.zeros(1, np.uint8)
    p = np.zeros(1, np.float32)
    assert L.bbe_bettors_create(k.ctypes.data, p.ctypes.data, 0, ctypes.byref(out)) == _bbe.EINVAL
    assert L.bbe_bettors_create(None, p.ctypes.data, 1, ctypes.byref(out)) == _bbe.EINVAL
    # a zeroed stand-in for a population handle: every case fails validation
    fake = np.zeros(64, np.uint64)
    h = ctypes.c_void_p(fake.ctypes.data)
    buf = ctypes.c_void_p(16)  # never dereferenced
    cases = [
        dict(n=0), dict(n=21), dict(L=0.0), dict(L=np.inf), dict(n_rows=0),
        dict(first_row=5, n_eval=6), dict(first_row=2**32 - 1, n_eval=2), dict(views=None, counts=None),
    ]
    for kw in cases:
        a = dict(n=3, L=100.0, n_rows=10, first_row=0, n_eval=10, views=buf, counts=buf)
        a.update(kw)
        rc = L.bbe_bettor_views(h, buf, a["n_rows"], a["n"], a["L"], 0, a["first_row"],
                                a["n_eval"], 1, a["views"], a["counts"], None)
        assert rc == _bbe.EINVAL, kw
    assert L.bbe_bettor_views(None, buf, 10, 3, 100.0, 0, 0, 1, 1, buf, buf, None) == _bbe.EINVAL
    assert L.bbe_bettor_views(h, None, 10, 3, 100.0, 0, 0, 1, 1, buf, buf, None) == _bbe.EINVAL
    race = _bbe.Race(np.array(GOOD, np.float32), 2000.0)
    for rows in (0, 2**20 + 2):
        assert L.bbe_race_trace(race.handle, None, 1, 0, 0, rows, buf, buf, None) == _bbe.EINVAL
    assert L.bbe_race_trace(race.handle, None, 1, 0, 0, 10, None, buf, None) == _bbe.EINVAL
    assert L.bbe_race_trace(None, None, 1, 0, 0, 10, buf, buf, None) == _bbe.EINVAL


def test_rp_views_reject_before_device_work(L):
    buf = ctypes.c_void_p(16)  # never dereferenced
    for n, stride in ((0, 20), (21, 21), (5, 4)):
        assert L.bbe_rp_views(buf, 10, n, stride, buf, buf, None) == _bbe.EINVAL
    assert L.bbe_rp_views(buf, -1, 5, 20, buf, buf, None) == _bbe.EINVAL
    assert L.bbe_rp_views(None, 10, 5, 20, buf, buf, None) == _bbe.EINVAL
    assert L.bbe_rp_views(buf, 10, 5, 20, None, None, None) == _bbe.EINVAL


def test_set_pace_rejects_and_leaves_the_race_unchanged(L):
    race = _bbe.Race(np.array(GOOD, np.float32), 2000.0)
    h = race.handle
    good_g = np.array([0.001, -0.001, 0.0], np.float32)
    good_t = np.array([100, 200, 0], np.float32)
    assert L.bbe_race_set_pace(h, good_g.ctypes.data, good_t.ctypes.data) == _bbe.OK
    bad = [
        ([np.nan, 0, 0], [1, 1, 1]), ([np.inf, 0, 0], [1, 1, 1]), ([0, 0, 0], [-1, 0, 0]),
        ([0, 0, 0], [1.5, 0, 0]), ([0, 0, 0], [2.0**25, 0, 0]),
        ([-0.01, 0, 0], [90, 0, 0]),  # 1 - 0.1 - 0.9 = 0 < 2^-10
    ]
    for g, t in bad:
        g = np.array(g, np.float32)
        t = np.array(t, np.float32)
        assert L.bbe_race_set_pace(h, g.ctypes.data, t.ctypes.data) == _bbe.EINVAL, (g, t)
        assert L.bbe_last_error().decode()
    assert L.bbe_race_set_pace(None, good_g.ctypes.data, good_t.ctypes.data) == _bbe.EINVAL
    assert L.bbe_race_set_pace(h, None, good_t.ctypes.data) == _bbe.EINVAL
    with pytest.raises(_bbe.BBEError):
        _bbe.Race(np.array([[5, 8, 1, 0.1, 2, -0.01, 90]] * 2, np.float32), 2000.0)
    with pytest.raises(_bbe.BBEError):
        _bbe.Race(np.zeros((3, 6), np.float32), 2000.0)


def test_pref_from_factors_host_function(L):
    """A host-only entry point (no device work): equals the oracle bit for
    bit, and rejects out-of-range values."""
    from oracle.factors import pref_from_factors as oracle_pref
    rng = np.random.default_rng(8)
    for n, F in ((1, 1), (5, 3), (20, 64), (7, 17)):
        f = rng.uniform(0, 1, F).astype(np.float32)
        p = rng.uniform(0, 1, (n, F)).astype(np.float32)
        w = rng.uniform(0, 0.6, (n, F)).astype(np.float32)
        np.testing.assert_array_equal(_bbe.pref_from_factors(f, p, w), oracle_pref(f, p, w))
    good = (np.float32([0.5]), np.float32([[0.5]]), np.float32([[0.5]]))
    for k, v in ((0, 1.5), (0, -0.1), (1, np.nan), (2, 1.0), (2, -0.5)):
        args = [a.copy() for a in good]
        args[k].flat[0] = v
        with pytest.raises(_bbe.BBEError):
            _bbe.pref_from_factors(*args)
    with pytest.raises(_bbe.BBEError):
        _bbe.pref_from_factors(np.zeros(65, np.float32), np.zeros((1, 65), np.float32),
                               np.zeros((1, 65), np.float32))
    with pytest.raises(_bbe.BBEError):  # underflow
        _bbe.pref_from_factors(np.zeros(64, np.float32), np.ones((1, 64), np.float32),
                               np.full((1, 64), 0.9999999, np.float32))


def test_mlp_load_rejects_bad_files(L, tmp_path):
    out = ctypes.c_void_p()
    assert L.bbe_mlp_load(str(tmp_path / "missing.bin").encode(), 8, ctypes.byref(out)) == _bbe.EINVAL
    bad_magic = tmp_path / "magic.bin"
    bad_magic.write_bytes(b"NOTANMLP" + (177940).to_bytes(4, "little") + bytes(4 * 177940))
    short = tmp_path / "short.bin"
    short.write_bytes(b"BBEMLP01" + (177940).to_bytes(4, "little") + bytes(4 * 1000))
    wrong_count = tmp_path / "count.bin"
    wrong_count.write_bytes(b"BBEMLP01" + (5).to_bytes(4, "little") + bytes(20))
    longer = tmp_path / "long.bin"
    longer.write_bytes(b"BBEMLP01" + (177940).to_bytes(4, "little") + bytes(4 * 177940 + 1))
    # training checkpoints: magic, count, step, then parameters and both
    # Adam moments; short files and invalid moments are rejected before any
    # device work
    np_ = 177940
    head = b"BBEMLP02" + np_.to_bytes(4, "little") + (7).to_bytes(8, "little")
    ck_short = tmp_path / "ck_short.bin"
    ck_short.write_bytes(head + bytes(4 * 2 * np_))
    ck_nan = tmp_path / "ck_nan.bin"
    m = np.zeros(3 * np_, np.float32)
    m[np_ + 5] = np.nan
    ck_nan.write_bytes(head + m.tobytes())
    ck_neg = tmp_path / "ck_neg.bin"
    m = np.zeros(3 * np_, np.float32)
    m[2 * np_ + 9] = -1e-3  # a second moment below zero
    ck_neg.write_bytes(head + m.tobytes())
    for f in (bad_magic, short, wrong_count, longer, ck_short, ck_nan, ck_neg):
        assert L.bbe_mlp_load(str(f).encode(), 8, ctypes.byref(out)) == _bbe.EINVAL, f
        assert L.bbe_last_error().decode()
    assert L.bbe_mlp_load(None, 8, ctypes.byref(out)) == _bbe.EINVAL
    assert L.bbe_mlp_save(None, b"/tmp/x") == _bbe.EINVAL
    assert L.bbe_mlp_save_checkpoint(None, b"/tmp/x") == _bbe.EINVAL


def test_prefix_batch_noalloc_rejects_before_device_work(L):
    """More requests than the fixed workspace holds, and NULL outputs, are
    rejected with BBE_EINVAL before anything touches a device."""
    race = _bbe.Race(np.array(GOOD, np.float32), 2000.0)
    for n, outs in ((_bbe.PREFIX_NOALLOC_MAX + 1, (1, 1, 1)), (2, (None, 1, 1))):
        arr, keep = _bbe._request_array([(race, None, 0, 1, i, 0) for i in range(n)])
        sims = np.zeros(n, np.uint32)
        targets = np.full(n, 100.0, np.float32)
        ptrs = [None if o is None else ctypes.c_void_p(16) for o in outs]
        rc = L.bbe_prefix_batch_noalloc(arr, sims.ctypes.data, targets.ctypes.data, n, 1,
                                        *ptrs, None)
        assert rc == _bbe.EINVAL
        msg = L.bbe_last_error().decode()
        assert ("static workspace" in msg) == (n > _bbe.PREFIX_NOALLOC_MAX), msg
        del keep
