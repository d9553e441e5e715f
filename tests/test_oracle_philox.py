"""Pins the oracle's Philox4x32-10 against rocRAND's implementation (an
independent implementation of the same published generator), run on the
host, and checks the draw conversion."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("pin") / "pin")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                    os.path.join(HERE, "native", "rocrand_philox_pin.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_oracle_philox_matches_rocrand(orc, rocrand_pin):
    rng = np.random.default_rng(1234)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] %= 2**30  # the rocRAND driver addresses low counter words through an offset
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    # a few structured counters (the layout the race model uses)
    ctr[:8] = [[t, s, 0, c] for t, s, c in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
                                            (329, 999_999, 4), (2**31, 7, 3), (5, 5, 2), (0, 0, 0)]]
    key[7] = [0xFFFFFFFF, 0xFFFFFFFF]
    lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([rocrand_pin], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in ln.split()] for ln in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    mine = np.array([orc.philox4x32_10(c, k) for c, k in zip(ctr, key)], dtype=np.uint64)
    assert ref.shape == (n, 4)
    np.testing.assert_array_equal(mine, ref)


def test_philox_output_is_not_trivial(orc):
    a = orc.philox4x32_10([0, 0, 0, 0], [0, 0])
    b = orc.philox4x32_10([1, 0, 0, 0], [0, 0])
    c = orc.philox4x32_10([0, 0, 0, 0], [1, 0])
    assert len({tuple(a), tuple(b), tuple(c)}) == 3


def test_draws_are_16_bit_halves(orc):
    """Competitor c's draw at tick t is one 16-bit half of the Philox word
    (c >> 1) & 3 of counter (t, sim, request, c >> 3): the high half for
    even c, the low half for odd c; u = k * 2^-16.  A race of 8 free
    competitors with lo = 1, hi = 1 + 2^-7 exposes u exactly in the first
    step: position 1 + 2^-7 * k * 2^-16 = 1 + k * 2^-23 is exact in float32
    for every k < 2^16, so all 16 bits of every draw are checked."""
    comp = np.array([[1.0, 1.0 + 2**-7, 1, 0, 0]] * 8, dtype=np.float32)
    seed, req, sim = 0x1234_5678_9ABC_DEF0, 77, 5
    t, pos, prev = orc.race_prefix(comp, 2000.0, seed, req, sim,
                                   target=np.nextafter(np.float32(0), np.float32(1)))
    w = orc.philox4x32_10([0, sim, req, 0], [seed & 0xFFFFFFFF, seed >> 32]).astype(np.uint64)
    k = np.array([(w[c >> 1] & 0xFFFF) if c & 1 else (w[c >> 1] >> 16) for c in range(8)])
    expect = 1.0 + k.astype(np.float64) * 2.0**-23
    assert t == 1
    np.testing.assert_array_equal(pos.astype(np.float64), expect)
    # competitors 8.. take the block of counter word c >> 3 = 1
    comp9 = np.array([[1.0, 1.0 + 2**-7, 1, 0, 0]] * 9, dtype=np.float32)
    _, pos9, _ = orc.race_prefix(comp9, 2000.0, seed, req, sim,
                                 target=np.nextafter(np.float32(0), np.float32(1)))
    w1 = orc.philox4x32_10([0, sim, req, 1], [seed & 0xFFFFFFFF, seed >> 32]).astype(np.uint64)
    assert pos9[8] == np.float32(1.0 + float(w1[0] >> 16) * 2.0**-23)
