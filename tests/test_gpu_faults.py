"""Error paths of the C ABI under injected faults (host side only: the
library's BBE_FAULT_INJECT hook makes a chosen device allocation or HIP
call fail without touching the GPU).  Each case runs in a fresh process
(tests/fault_cases.py) and checks that the failing call returns BBE_ENOMEM
or BBE_EDEVICE with a message naming the failed step, that nothing is left
half-built (the next identical call succeeds), and that the results
computed after the failures equal those of an undisturbed run."""
import json
import os
import subprocess
import sys

import pytest

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
ENOMEM, EDEVICE = -2, -3


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _run(case, spec):
    announce(f"fault case {case}: BBE_FAULT_INJECT={spec!r}")
    env = dict(os.environ, BBE_FAULT_INJECT=spec)
    p = subprocess.run([sys.executable, os.path.join(HERE, "fault_cases.py"), case], env=env,
                       capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-3000:]
    line = [ln for ln in p.stdout.splitlines() if ln.startswith("{")][-1]
    res = json.loads(line)
    assert all(res["checks"].values()), res
    return res["outcomes"]


def _expect(outcomes, want):
    """want: one (code, message fragment) per call; code 0 = success."""
    assert len(outcomes) == len(want), outcomes
    for (code, msg), (wc, frag) in zip(outcomes, want):
        assert code == wc, (outcomes, want)
        if wc:
            assert frag in msg, (msg, frag)
            if wc == EDEVICE:
                assert "hipErrorLaunchFailure" in msg, msg


# Counted HIP calls per entry point, in order: bbe_race_sim: clear the win
# counts, clear the step count, launch; bbe_win_probs: launch.
def test_race_sim_device_faults(torch):
    _expect(_run("race_sim", "device:1,4,8"),
            [(EDEVICE, "zeroing win_counts"), (EDEVICE, "launching race_mc_kernel"), (0, ""),
             (EDEVICE, "launching win_probs_kernel"), (0, ""), (0, "")])


# Plan creation without autotuning allocates the request table, the queue
# and the work list, and makes five counted calls: copy the request table,
# create the capture stream, copy the work list, begin the capture,
# instantiate the graph; each launch is one more.
def test_plan_allocation_faults(torch):
    msg_table = "device allocation of the request table failed"
    _expect(_run("plan", "alloc:1,3,6"),
            [(ENOMEM, msg_table), (ENOMEM, msg_table),
             (ENOMEM, "device allocation of the work list failed"), (0, ""), (0, ""), (0, "")])


def test_plan_device_faults(torch):
    _expect(_run("plan", "device:1,3,6,10,15,21"),
            [(EDEVICE, "copying the request table"), (EDEVICE, "creating the capture stream"),
             (EDEVICE, "copying the work list"), (EDEVICE, "beginning graph capture"),
             (EDEVICE, "instantiating the graph"), (0, ""),
             (EDEVICE, "launching the plan graph"), (0, "")])


# A network with max_batch 8 makes 19 device allocations (parameters, Adam
# moments, gradient, weight copies, activations, work tiles).
def test_mlp_allocation_faults(torch):
    msg = "device allocation of the network failed"
    _expect(_run("mlp", "alloc:1,3,22"),
            [(ENOMEM, msg), (ENOMEM, msg), (ENOMEM, msg), (0, ""), (0, ""), (0, "")])


def test_mlp_device_faults(torch):
    _expect(_run("mlp", "device:1,3"),
            [(EDEVICE, "initialising the network"), (0, ""),
             (EDEVICE, "launching the forward pass"), (0, "")])


def test_bettors_faults(torch):
    msg = "device allocation of 300 bettors failed"
    _expect(_run("bettors", "alloc:1,3,6"),
            [(ENOMEM, msg), (ENOMEM, msg), (ENOMEM, msg), (0, ""), (0, ""), (0, "")])
    _expect(_run("bettors", "device:1,3"),
            [(EDEVICE, "copying the bettors"), (0, ""),
             (EDEVICE, "launching bettor_views_kernel"), (0, "")])


def test_prefix_batch_faults(torch):
    _expect(_run("prefix", "alloc:1"),
            [(ENOMEM, "device allocation failed"), (0, ""), (0, ""), (0, "")])
    _expect(_run("prefix", "device:1,3"),
            [(EDEVICE, "in-play state batch"), (EDEVICE, "in-play state batch"), (0, ""),
             (0, "")])


def test_noalloc_entry_point_allocates_nothing_and_recovers(torch):
    """The allocation-free variant makes no device allocation (the first
    one of the process is the reference call's), and recovers from device
    faults in its staging copy and its launch."""
    _expect(_run("prefix_noalloc", "alloc:1"),
            [(0, ""), (0, ""), (0, ""), (ENOMEM, "device allocation failed"), (0, "")])
    _expect(_run("prefix_noalloc", "device:1,3"),
            [(EDEVICE, "staging the request descriptors"), (EDEVICE, "in-play state batch"),
             (0, ""), (0, "")])
