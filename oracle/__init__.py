"""Plain CPU oracle of the BBE race model and of the surrogate network.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library never imports, links or calls it, and it shares no code with the
GPU path.

Contents
--------
``race_oracle.c``  scalar C implementation of the race model (paper
                   Section 3, Eq. 1) with its own Philox4x32-10; built into
                   ``liborc.so`` by :func:`build`.
``enumerate.py``   independent pure-Python exact enumeration of tiny races.
``twocomp.py``     exact law of a two-competitor race by dynamic programming.
``mlp.py``         float64 numpy reference of the surrogate network and of
                   the state encoding fed to it.
``orders.py``      finish-position counts and finish-order PMF.
``bettors.py``     the cheap in-play bettor rules (LinEx, LW, UD, ZI).

Functions here take and return numpy arrays.  Competitor parameters are an
``[n, 5]`` float32 array of ``(lo, hi, pref, rho, theta)`` rows, or ``[n, 7]``
with the time term ``(gamma, tau)`` of the responsiveness appended
(``[n, 5]`` means gamma = 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "race_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

OK = 0
EINVAL = -1
MAX_N = 20


def build(force: bool = True) -> str:
    """Compile ``liborc.so`` with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u32, u64, i32, f32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_float
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox4x32_10.restype = None
        L.orc_race_sim.argtypes = [i32, f32, P, u32, P, P, u32, u32, u64, u32, i32, u32,
                                   P, P, P, i32]
        L.orc_race_sim.restype = i32
        L.orc_race_draws.argtypes = [i32, f32, P, u32, P, P, i32, i32, i32, P, P, P, P]
        L.orc_race_draws.restype = i32
        L.orc_race_prefix.argtypes = [i32, f32, P, u32, P, P, u64, u32, u32, f32, P, P, P]
        L.orc_race_prefix.restype = i32
        L.orc_race_trace.argtypes = [i32, f32, P, u32, P, P, u64, u32, u32, u32, P, P]
        L.orc_race_trace.restype = i32
        L.orc_win_probs.argtypes = [P, i32, P]
        L.orc_win_probs.restype = i32
        L.orc_tick_limit.restype = u32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _comp(comp) -> np.ndarray:
    """Competitor rows as the C oracle takes them: [n, 7] float32."""
    c = np.asarray(comp, dtype=np.float32)
    if c.ndim != 2 or c.shape[1] not in (5, 7):
        raise OracleError("competitor rows must have 5 or 7 columns")
    if c.shape[1] == 5:
        c = np.concatenate([c, np.zeros((c.shape[0], 2), np.float32)], axis=1)
    return np.ascontiguousarray(c)


class OracleError(ValueError):
    pass


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block for counter ``ctr`` (4 x u32) and key (2 x u32)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def race_sim(comp, L, n_sims, seed, request=0, state=None, sim_begin=0, stop_after=None,
             levels=0, want_orders=True, threads=1):
    """Monte-Carlo over sims [sim_begin, sim_begin+n_sims).

    ``state`` is ``None`` (start of race) or ``(tick, pos[n], prev[n])``.
    Returns ``(orders [n_sims, n] uint8 or None, wins [n] uint64,
    competitor_steps int)``.
    """
    comp = _comp(comp)
    n = comp.shape[0]
    if stop_after is None:
        stop_after = n
    t0, pos, prev = 0, None, None
    if state is not None:
        t0, pos, prev = int(state[0]), _f32(state[1]), _f32(state[2])
    orders = np.empty((n_sims, n), dtype=np.uint8) if want_orders else None
    wins = np.zeros(n, dtype=np.uint64)
    steps = np.zeros(1, dtype=np.uint64)
    rc = lib().orc_race_sim(n, float(L), _ptr(comp), t0, _ptr(pos), _ptr(prev), sim_begin,
                            n_sims, seed, request, stop_after, levels, _ptr(orders),
                            _ptr(wins), _ptr(steps), threads)
    if rc != OK:
        raise OracleError(f"orc_race_sim rejected the arguments (rc={rc})")
    return orders, wins, int(steps[0])


def race_draws(comp, L, draws, state=None, stop_after=None, return_used=False,
               return_trace=False):
    """Run ``draws.shape[0]`` races driven by explicit draws ``[seq, tick, n]``.

    Returns the orders, plus (on request) the consumed-draw mask and the
    positions after every tick (``[seq, tick, n]``, NaN past the end)."""
    comp = _comp(comp)
    n = comp.shape[0]
    if stop_after is None:
        stop_after = n
    draws = np.ascontiguousarray(draws, dtype=np.float32)
    n_seq, max_ticks, n2 = draws.shape
    assert n2 == n
    t0, pos, prev = 0, None, None
    if state is not None:
        t0, pos, prev = int(state[0]), _f32(state[1]), _f32(state[2])
    orders = np.empty((n_seq, n), dtype=np.uint8)
    used = np.zeros(draws.shape, dtype=np.uint8) if return_used else None
    trace = np.full(draws.shape, np.nan, dtype=np.float32) if return_trace else None
    rc = lib().orc_race_draws(n, float(L), _ptr(comp), t0, _ptr(pos), _ptr(prev), stop_after,
                              n_seq, max_ticks, _ptr(draws), _ptr(orders), _ptr(used),
                              _ptr(trace))
    if rc != OK:
        raise OracleError(f"orc_race_draws rejected the arguments (rc={rc})")
    out = [orders]
    if return_used:
        out.append(used)
    if return_trace:
        out.append(trace)
    return out[0] if len(out) == 1 else tuple(out)


def race_prefix(comp, L, seed, request, sim, target, state=None):
    """Advance one simulated race until the leader is at ``target``; returns
    the in-play state ``(tick, pos, prev)``."""
    comp = _comp(comp)
    n = comp.shape[0]
    t0, pos, prev = 0, None, None
    if state is not None:
        t0, pos, prev = int(state[0]), _f32(state[1]), _f32(state[2])
    t_out = np.zeros(1, dtype=np.uint32)
    p_out = np.zeros(n, dtype=np.float32)
    s_out = np.zeros(n, dtype=np.float32)
    rc = lib().orc_race_prefix(n, float(L), _ptr(comp), t0, _ptr(pos), _ptr(prev), seed,
                               request, sim, float(target), _ptr(t_out), _ptr(p_out),
                               _ptr(s_out))
    if rc != OK:
        raise OracleError(f"orc_race_prefix rejected the arguments (rc={rc})")
    return int(t_out[0]), p_out, s_out


def race_trace(comp, L, seed, request, sim, max_rows, state=None):
    """Positions ``[rows, n]`` of one simulated race tick by tick, from the
    state (row 0) until just before the first tick in which a competitor
    would reach the line, or ``max_rows`` rows."""
    comp = _comp(comp)
    n = comp.shape[0]
    t0, pos, prev = 0, None, None
    if state is not None:
        t0, pos, prev = int(state[0]), _f32(state[1]), _f32(state[2])
    trace = np.zeros((max_rows, n), dtype=np.float32)
    rows = np.zeros(1, dtype=np.uint32)
    rc = lib().orc_race_trace(n, float(L), _ptr(comp), t0, _ptr(pos), _ptr(prev), seed,
                              request, sim, int(max_rows), _ptr(trace), _ptr(rows))
    if rc != OK:
        raise OracleError(f"orc_race_trace rejected the arguments (rc={rc})")
    return trace[: int(rows[0])].copy()


def win_probs(wins) -> np.ndarray:
    w = np.ascontiguousarray(wins, dtype=np.uint64)
    p = np.zeros(w.shape[0], dtype=np.float64)
    rc = lib().orc_win_probs(_ptr(w), w.shape[0], _ptr(p))
    if rc != OK:
        raise OracleError("orc_win_probs rejected the arguments")
    return p


def tick_limit() -> int:
    return int(lib().orc_tick_limit())
