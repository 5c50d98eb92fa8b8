"""The cooperative large-node path, built for the CPU, against the oracle.

tests/host/wave_host_check.cpp compiles bt_wave.hpp and bt_device.hpp with g++
(BT_HOST_DEBUG: a wavefront of any width emulated lane by lane) and prices
whole trees level by level with every node sent through the cooperative path
(threshold 0).  Seeded random puts, calls and bull spreads (American, European
and cost-at-t=0 variants) must give the oracle's ask, bid and breakpoint
counts bit for bit, and with tangents the oracle's Greeks bit for bit, for
64 emulated lanes (the GPU's wavefront) and for 2 or 3 lanes (tiles of a few
positions, so that every tile boundary case occurs in small trees)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "wave_host_check.cpp")
CSRC = os.path.join(ROOT, "paper_1110_2477_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path_factory.mktemp("hostwave") / "wave_host_check")
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC, "-o", exe, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _cases(seed, n, n_max):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(n):
        pay = int(rng.integers(0, 3))
        S0 = 100 * np.exp(0.2 * rng.standard_normal())
        K = S0 * rng.uniform(0.8, 1.2)
        K2 = K * rng.uniform(1.05, 1.3)
        sig, T, R = rng.uniform(0.1, 0.6), rng.uniform(0.1, 2), rng.uniform(0, 0.08)
        k = rng.choice([0.0, rng.uniform(0, 0.02), rng.uniform(0, 0.1)])
        N = int(rng.integers(1, n_max))
        fl = int(rng.choice([0, 0, 0, 1, 2]))
        cases.append((float(S0), float(K), float(K2), float(R), float(sig), float(T), float(k), N, pay, fl))
    return cases


def _run(exe, cases, grad, lanes, split=False):
    inp = "\n".join(" ".join(repr(x) if j < 7 else str(int(x)) for j, x in enumerate(c)) for c in cases) + "\n"
    r = subprocess.run([exe, "0", "1" if grad else "0", str(lanes), "1" if split else "0"], input=inp,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = r.stdout.strip().split("\n")
    assert len(out) == len(cases)
    return out, r.stderr


def _oracle(c, grad):
    return oracle.price(c[0], c[1], c[3], c[4], c[5], c[6], c[7], payoff=c[8], K2=c[2], flags=c[9], grad=grad)


@pytest.mark.parametrize("lanes,split", [(64, False), (3, False), (64, True), (3, True), (2, True)])
def test_cooperative_path_prices_match_oracle(harness, lanes, split):
    # split: the envelope's final merge in two halves, the upper half from an
    # unknown arriving slope, as the helper wave of a workgroup runs it
    cases = _cases(seed=101 + lanes, n=40, n_max=140)
    out, err = _run(harness, cases, grad=False, lanes=lanes, split=split)
    for c, line in zip(cases, out):
        f = line.split()
        o = _oracle(c, grad=False)
        assert int(f[0]) == 0, c
        assert float.fromhex(f[1]) == o["ask"] and float.fromhex(f[2]) == o["bid"], (c, f[:3], o)
        assert (int(f[3]), int(f[4]), int(f[5]), int(f[6])) == (
            o["bp_total_ask"], o["bp_total_bid"], o["bp_max_ask"], o["bp_max_bid"]), c
    # the envelope's halves were merged from their schedule
    assert "envelope merges: scheduled" in err
    assert int(err.split("scheduled")[1].split(",")[0]) > 0
    if split and lanes < 64:
        # merges were split, and some upper half's first point was dropped
        n_split, n_drop = (int(x) for x in err.split("split merges:")[1].split("\n")[0].split(", dropped"))
        assert n_split > 0 and n_drop > 0, (n_split, n_drop)


@pytest.mark.parametrize("lanes", [64, 2])
def test_cooperative_path_tangents_match_oracle(harness, lanes):
    cases = _cases(seed=201 + lanes, n=24, n_max=90)
    out, _ = _run(harness, cases, grad=True, lanes=lanes)
    for c, line in zip(cases, out):
        f = line.split()
        o = _oracle(c, grad=True)
        assert int(f[0]) == 0, c
        assert float.fromhex(f[1]) == o["ask"] and float.fromhex(f[2]) == o["bid"], c
        ga = np.array([float.fromhex(x) for x in f[7:11]])
        gb = np.array([float.fromhex(x) for x in f[11:15]])
        assert np.array_equal(ga, o["grad_ask"]) and np.array_equal(gb, o["grad_bid"]), (c, ga, gb, o)


def test_cooperative_path_every_payoff_shape(harness):
    # cash-settled puts and calls, bear spreads and straddles as well
    from paper_1110_2477_amd import workloads as W
    b = W.variants_book(28, seed=104, n_max=120)
    cases = [(float(p["S0"]), float(p["K"]), float(p["K2"]), float(p["R"]), float(p["sigma"]), float(p["T"]),
              float(p["k"]), int(p["N"]), int(p["payoff"]), int(p["flags"])) for p in b]
    out, _ = _run(harness, cases, grad=True, lanes=64)
    for c, line in zip(cases, out):
        f = line.split()
        o = _oracle(c, grad=True)
        assert int(f[0]) == 0, c
        assert float.fromhex(f[1]) == o["ask"] and float.fromhex(f[2]) == o["bid"], c
        assert (int(f[3]), int(f[4]), int(f[5]), int(f[6])) == (
            o["bp_total_ask"], o["bp_total_bid"], o["bp_max_ask"], o["bp_max_bid"]), c
        ga = np.array([float.fromhex(x) for x in f[7:11]])
        gb = np.array([float.fromhex(x) for x in f[11:15]])
        assert np.array_equal(ga, o["grad_ask"]) and np.array_equal(gb, o["grad_bid"]), c

