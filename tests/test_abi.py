"""The C-ABI library loads and exports what include/bt.h declares; host-side
logic that needs no GPU (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "bt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bt.LIB_PATH):
        from paper_1110_2477_amd import build
        build.build()
    return bt.lib()


def test_every_declared_function_is_exported(lib):
    names = header_functions()
    assert set(names) == set(bt.ABI_FUNCTIONS)
    for name in names:
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_version_and_errors(lib):
    assert bt.bt_version() == 10000
    assert bt.strerror(0) == "success"
    assert "invalid" in bt.strerror(-1)
    assert bt.strerror(-99) == "unknown error"


def test_struct_sizes_match_header():
    src = open(os.path.join(ROOT, "include", "bt.h")).read()
    assert "double S0, K, K2, R, sigma, T, k;" in src
    assert W.PARAMS_DTYPE.itemsize == 7 * 8 + 4 * 4
    assert W.RESULT_DTYPE.itemsize == 3 * 8 + 2 * 8 + 4 * 4
    assert W.GRAD_DTYPE.itemsize == 8 * 8


def test_model_constants_match_oracle_bitwise(lib):
    # The tree constants (Section 4.1) are derived on the host by the
    # library and, independently, by the oracle; both use the same formulas,
    # so they agree to the bit.
    hard = W.single_put_n100().repeat(4)
    # sigma = exponent with T = N = 1: arguments whose libm exp is not the
    # nearest binary64 number
    for i, h in enumerate(["0x1.a056d88f0ced3p-8", "0x1.88ab8b85f2710p-9", "0x1.983139ccee7acp-7",
                           "0x1.6c15d3740474dp-9"]):
        hard[i]["sigma"], hard[i]["T"], hard[i]["N"], hard[i]["R"] = float.fromhex(h), 1.0, 1, 0.0
    for b in (W.single_put_n100(), W.paper_grid(1500)[:3], W.mixed_book(16, seed=9), hard,
              W.stress_book(2000, seed=12), W.mixed_book(2000, seed=13)):
        for p in b:
            c = bt.bt_model_constants(p)
            _, o = oracle.model_table(p["S0"], p["sigma"], p["R"], p["T"], int(p["N"]))
            for key in ("u", "d", "r", "rho", "p"):
                assert c[key] == o[key], key


def test_invalid_parameters_are_rejected_on_the_host(lib):
    good = W.single_put_n100()[0]
    for field, value in (("N", 0), ("k", 1.0), ("sigma", -0.1), ("S0", 0.0), ("T", np.nan),
                         ("payoff", 7), ("flags", 8)):
        p = good.copy()
        p[field] = value
        with pytest.raises(bt.BtError) as e:
            bt.bt_model_constants(p)
        assert e.value.code == bt.BT_EINVAL
    p = good.copy()
    p["R"], p["sigma"], p["N"] = 5.0, 0.01, 2   # r > u: the tree has arbitrage
    with pytest.raises(bt.BtError):
        bt.bt_model_constants(p)


def test_workload_generators_are_seeded_and_shaped():
    a, b = W.mixed_book(64, seed=3), W.mixed_book(64, seed=3)
    assert a.tobytes() == b.tobytes()
    m = W.mixed_book(4096)
    assert m["N"].min() >= 200 and m["N"].max() <= 2000
    frac = np.bincount(m["payoff"], minlength=3) / len(m)
    assert abs(frac[0] - 0.4) < 0.03 and abs(frac[1] - 0.4) < 0.03 and abs(frac[2] - 0.2) < 0.03
    bull = m["payoff"] == W.BULL
    assert np.all(m["K2"][bull] > m["K"][bull])
    s = W.stress_book(2048)
    assert s["N"].min() >= 64 and s["N"].max() <= 8192
    g = W.paper_grid(1500)
    assert len(g) == 24 and set(g["N"]) == {1500}
