"""The oracle built with the address and undefined-behaviour sanitizers
(gcc -fsanitize=address,undefined, stop at the first report, leak check at
exit) runs the Monte-Carlo, the in-play state generator, the trace and the
win probabilities on several races -- from the start, in play, tied
identical competitors, one competitor -- without a report, and computes
exactly what the plain build computes (no GPU)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as orc
from paper_2108_02419_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
L = 2000.0


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "oracle_sanitize_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fno-fast-math", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wno-unknown-pragmas", "-o", exe,
           os.path.join(HERE, "native", "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "race_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return exe, d


def _run(driver, comp, state, sim_begin, n_sims, seed, request, stop_after, target, max_rows):
    exe, d = driver
    comp = orc._comp(comp)  # [n, 7]: the time-term columns zero unless given
    n = comp.shape[0]
    t0, pos, prev = (0, np.zeros(n, np.float32), np.zeros(n, np.float32)) if state is None \
        else (state[0], np.asarray(state[1], np.float32), np.asarray(state[2], np.float32))
    blob = b"".join([np.int32(n).tobytes(), np.float32(L).tobytes(), comp.tobytes(),
                     np.uint32(t0).tobytes(), np.int32(state is not None).tobytes(),
                     pos.tobytes(), prev.tobytes(), np.uint32(sim_begin).tobytes(),
                     np.uint32(n_sims).tobytes(), np.uint64(seed).tobytes(),
                     np.uint32(request).tobytes(), np.int32(stop_after).tobytes(),
                     np.float32(target).tobytes(), np.uint32(max_rows).tobytes()])
    fin, fout = str(d / "in.bin"), str(d / "out.bin")
    open(fin, "wb").write(blob)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    p = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0 and "runtime error" not in p.stderr \
        and "ERROR: AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    raw = open(fout, "rb").read()
    o = 0

    def take(dtype, count):
        nonlocal o
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=o)
        o += a.nbytes
        return a

    out = {}
    out["sim_rc"] = int(take(np.int32, 1)[0])
    out["orders"] = take(np.uint8, n_sims * n).reshape(n_sims, n)
    out["wins"] = take(np.uint64, n)
    out["steps"] = int(take(np.uint64, 1)[0])
    out["prefix_rc"] = int(take(np.int32, 1)[0])
    out["tick"] = int(take(np.uint32, 1)[0])
    out["pos"] = take(np.float32, n)
    out["prev"] = take(np.float32, n)
    out["trace_rc"] = int(take(np.int32, 1)[0])
    rows = int(take(np.uint32, 1)[0])
    out["trace"] = take(np.float32, rows * n).reshape(rows, n)
    out["probs_rc"] = int(take(np.int32, 1)[0])
    out["probs"] = take(np.float64, n)
    assert o == len(raw)
    return out


def _cases():
    c5 = inputs.competitor_params(np.random.default_rng(1), 5)
    c20 = inputs.competitor_params(np.random.default_rng(2), 20)
    st20 = orc.race_prefix(c20, L, 3, 0x80000001, 0, np.float32(700.0))
    same = np.tile(np.float32([[6.5, 6.5, 1.0, 0.0, 2.0]]), (4, 1))  # identical, deterministic
    c1 = inputs.competitor_params(np.random.default_rng(3), 1)
    blocking = inputs.competitor_params(np.random.default_rng(4), 12)
    blocking[:, 4] = np.float32(6.0)  # long blocking chains
    paced = inputs.pace_params(np.random.default_rng(5),
                               inputs.competitor_params(np.random.default_rng(5), 8))
    return [("start_n5", c5, None, 0, 700, 1, 0, 5, 900.0, 400),
            ("inplay_n20_winner", c20, st20, 1000, 300, 3, 2, 1, 1500.0, 400),
            ("ties_n4", same, None, 0, 64, 5, 0, 4, 1000.0, 400),
            ("one_n1", c1, None, 2**32 - 70, 70, 6, 9, 1, 1500.0, 500),
            ("blocking_n12", blocking, None, 0, 200, 7, 4, 12, 600.0, 120),
            ("time_term_n8", paced, None, 0, 300, 8, 5, 3, 800.0, 300)]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_sanitized_oracle_matches_plain_build(driver, case):
    name, comp, state, begin, n_sims, seed, request, stop, target, max_rows = case
    got = _run(driver, comp, state, begin, n_sims, seed, request, stop, target, max_rows)
    assert got["sim_rc"] == got["prefix_rc"] == got["trace_rc"] == got["probs_rc"] == 0
    o, w, s = orc.race_sim(comp, L, n_sims, seed, request=request, state=state,
                           sim_begin=begin, stop_after=stop)
    np.testing.assert_array_equal(got["orders"], o)
    np.testing.assert_array_equal(got["wins"], w)
    assert got["steps"] == s
    t, p, v = orc.race_prefix(comp, L, seed, request, 0, np.float32(target), state=state)
    assert got["tick"] == t
    np.testing.assert_array_equal(got["pos"], p)
    np.testing.assert_array_equal(got["prev"], v)
    np.testing.assert_array_equal(got["trace"],
                                  orc.race_trace(comp, L, seed, request, 0, max_rows, state=state))
    np.testing.assert_array_equal(got["probs"], orc.win_probs(w))
