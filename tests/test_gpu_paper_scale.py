"""Parity at the paper's scale against stored oracle results
(tests/golden/paper_scale.json, written by tests/golden/make_paper_scale.py,
which calls only the oracle):

* the N = 20000 put (ask, bid, price0 and breakpoint counts);
* the 32 options of the Greeks book (N 500..1500) of the finite-difference
  check: prices, counts and the Greeks against the oracle's forward-mode
  derivatives, through the device-resident batch entry point;
* a seeded 32-option sample of the stress book spanning N 64..8192, with 8
  calls and bull spreads at N >= 4000 and k >= 1 %.

Bar: prices within 1e-10 relative, counts equal, Greeks within 1e-9
relative (floor 1)."""
import json
import os

import numpy as np
import pytest

import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

from test_gpu_parity import rel, say

pytestmark = pytest.mark.gpu
RTOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_scale.json")
COUNTS = ("bp_total_ask", "bp_total_bid", "bp_max_ask", "bp_max_bid")


@pytest.fixture(scope="module")
def golden():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bt.lib()
    with open(GOLDEN) as f:
        yield json.load(f)
    bt.bt_shutdown()


def _book(cases):
    return W.book([c["params"] for c in cases])


def _compare(b, res, cases, sides=("ask", "bid")):
    worst = 0.0
    for i, c in enumerate(cases):
        o = c["oracle"]
        assert res[i]["status"] == 0, (i, res[i]["status"])
        for key in sides + ("price0",):
            e = rel(res[i][key], o[key])
            worst = max(worst, e)
            assert e <= RTOL, (i, key, res[i][key], o[key], b[i])
        for key in COUNTS:
            if key in o:
                assert int(res[i][key]) == o[key], (i, key, int(res[i][key]), o[key], b[i])
    return worst


def test_long_put_n20000_matches_the_oracle(golden):
    cases = golden["long_put"]
    b = _book(cases)
    say("case: put N=20000, k=1% (book)")
    res = bt.price_book(b)
    w = _compare(b, res, cases)
    say(f"  ask {res[0]['ask']!r} bid {res[0]['bid']!r}, worst rel err {w:.3g}, "
        f"max breakpoints {res[0]['bp_max_ask']}/{res[0]['bp_max_bid']}")


def test_stress_sample_to_n8192_matches_the_oracle(golden):
    cases = golden["stress_sample"]
    b = _book(cases)
    heavy = int(np.sum((b["N"] >= 4000) & (b["k"] >= 0.01) & (b["payoff"] != W.PUT)))
    say(f"case: stress sample, {len(b)} options, N {b['N'].min()}..{b['N'].max()}, {heavy} costly calls/bull "
        f"spreads with N >= 4000")
    assert heavy >= 8
    res = bt.price_book(b)
    w = _compare(b, res, cases)
    say(f"  worst rel err {w:.3g}; largest node {int(res['bp_max_bid'].max())} breakpoints")


def test_greeks_book_fd_subset_matches_oracle_tangents(golden):
    import torch
    cases = golden["greeks_fd32"]
    b = _book(cases)
    say(f"case: Greeks of the 32 FD options (N {b['N'].min()}..{b['N'].max()}) via bt_price_grad_batch")
    out, g = bt.price_batch(bt.params_tensor(b), max_N=int(b["N"].max()), grad=True)
    torch.cuda.synchronize()
    res, gr = bt.as_results(out), bt.as_grads(g)
    _compare(b, res, cases)
    worst = 0.0
    for i, c in enumerate(cases):
        for side in ("ask", "bid"):
            ad = np.array([gr[i][f"{side}_d{k}"] for k in ("S0", "sigma", "R", "k")])
            ref = np.array(c["oracle"]["grad_" + side])
            err = float(np.max(np.abs(ad - ref) / np.maximum(1.0, np.abs(ref))))
            worst = max(worst, err)
            assert err <= 1e-9, (i, side, ad, ref)
    say(f"  worst Greek difference {worst:.3g}")
