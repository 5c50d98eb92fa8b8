"""The reverse sweep of the Greeks (bt_adjoint.hpp), built for the CPU,
against the oracle's forward-mode derivatives.

tests/host/adjoint_host_check.cpp compiles bt_adjoint.hpp and bt_device.hpp
with g++ and runs, for whole trees, the schedule of the GPU's adjoint kernel:
a forward pass keeping every s-th level (s = ceil(sqrt(N+2))) as a
checkpoint, then the reverse pass from the root, segment by segment,
recomputing each segment from its upper checkpoint and stepping every node
back through the taped recomputation of its update.  Seeded random puts,
calls and bull spreads (American, European and cost-at-t=0 variants, costs up
to 10 %) and high-cost trees with hundreds of breakpoints per node must give
the oracle's prices and breakpoint counts bit for bit and its derivatives
d(ask, bid)/d(S0, sigma, R, k) within 1e-9 (relative, floor 1): the two
methods are independent (tangents carried forward through the C oracle
against a tape read backwards here) and agree up to rounding."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from test_host_wave_path import _cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "adjoint_host_check.cpp")
CSRC = os.path.join(ROOT, "paper_1110_2477_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path_factory.mktemp("hostadj") / "adjoint_host_check")
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           "-o", exe, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, cases):
    inp = "\n".join(" ".join(repr(x) if j < 7 else str(int(x)) for j, x in enumerate(c)) for c in cases) + "\n"
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    out = r.stdout.strip().split("\n")
    assert len(out) == len(cases)
    return out


def _check(cases, out):
    worst = 0.0
    for c, line in zip(cases, out):
        f = line.split()
        assert int(f[0]) == 0, c
        o = oracle.price(c[0], c[1], c[3], c[4], c[5], c[6], c[7], payoff=c[8], K2=c[2], flags=c[9], grad=True)
        assert float.fromhex(f[1]) == o["ask"] and float.fromhex(f[2]) == o["bid"], (c, f[:3], o)
        assert (int(f[3]), int(f[4]), int(f[5]), int(f[6])) == (
            o["bp_total_ask"], o["bp_total_bid"], o["bp_max_ask"], o["bp_max_bid"]), c
        g = np.array([float.fromhex(x) for x in f[7:15]])
        ref = np.concatenate([o["grad_ask"], o["grad_bid"]])
        err = float(np.max(np.abs(g - ref) / np.maximum(1.0, np.abs(ref))))
        worst = max(worst, err)
        assert err <= 1e-9, (c, g, ref)
    return worst


def test_reverse_sweep_matches_oracle_tangents_on_random_trees(harness):
    cases = _cases(seed=301, n=40, n_max=160)
    _check(cases, _run(harness, cases))


def test_reverse_sweep_on_high_cost_trees(harness):
    # 2k / (sigma sqrt(dt)) well above 1: hundreds of breakpoints per node,
    # and N + 2 a perfect square (checkpoints every sqrt(N+2) levels exactly)
    cases = [(100.0, 100.0, 0.0, 0.03, 0.15, 0.5, 0.08, 223, 1, 0),
             (100.0, 95.0, 105.0, 0.03, 0.15, 0.5, 0.05, 254, 2, 0),
             (100.0, 100.0, 0.0, 0.05, 0.3, 1.0, 0.01, 300, 1, 2),
             (100.0, 110.0, 0.0, 0.05, 0.3, 1.0, 0.01, 198, 0, 1),
             (100.0, 100.0, 0.0, 0.05, 0.2, 1.0, 0.005, 1, 0, 0),
             (100.0, 100.0, 0.0, 0.05, 0.2, 1.0, 0.005, 2, 1, 0)]
    _check(cases, _run(harness, cases))
