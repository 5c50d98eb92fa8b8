"""Reverse-mode Greeks (bt_price_adjoint_batch: the checkpointed reverse
sweep) against the oracle's forward-mode derivatives, against the library's
own forward-mode Greeks, and against central finite differences of the GPU
prices.  Prices and breakpoint counts are the batch entry point's bits."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

from test_gpu_greeks import _fd_check, grads_of
from test_gpu_parity import say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_scale.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bt.lib()
    yield
    bt.bt_shutdown()


def adjoint(b, max_N=None):
    import torch
    max_N = int(b["N"].max()) if max_N is None else max_N
    out, g = bt.price_batch(bt.params_tensor(b), max_N=max_N, grad=True, mode="adjoint")
    torch.cuda.synchronize()
    return bt.as_results(out), bt.as_grads(g)


def _rel(ad, ref):
    return float(np.max(np.abs(ad - ref) / np.maximum(1.0, np.abs(ref))))


def test_adjoint_matches_oracle_and_forward_mode_on_random_trees():
    import torch
    b = W.random_small(64, seed=91, n_max=200)
    bad = W.single_put_n100().repeat(2)
    bad[0]["N"] = 0      # invalid
    bad[1]["N"] = 220    # above max_N
    b = np.concatenate([b, bad])
    say(f"case: reverse-mode Greeks of {len(b)} options (random, invalid, N above max_N)")
    res, g = adjoint(b, max_N=200)
    assert res[-2]["status"] == bt.BT_EINVAL and res[-1]["status"] == bt.BT_EINVAL
    assert np.isnan(g[-1]["ask_dS0"]) and np.isnan(res[-1]["bid"])
    b = b[:-2]
    res, g = res[:-2], g[:-2]
    out = bt.price_batch(bt.params_tensor(b), max_N=200)
    fo, fg = bt.price_batch(bt.params_tensor(b), max_N=200, grad=True)
    torch.cuda.synchronize()
    ref_res, fwd = bt.as_results(out), bt.as_grads(fg)
    assert res.tobytes() == ref_res.tobytes()
    worst_o = worst_f = 0.0
    for i in range(len(b)):
        o = oracle.price_params(b[i], grad=True)
        for side in ("ask", "bid"):
            ad = grads_of(g[i], side)
            eo, ef = _rel(ad, o["grad_" + side]), _rel(ad, grads_of(fwd[i], side))
            worst_o, worst_f = max(worst_o, eo), max(worst_f, ef)
            assert eo <= 1e-9, (i, side, ad, o["grad_" + side], b[i])
            assert ef <= 1e-9, (i, side, ad, grads_of(fwd[i], side))
    say(f"  worst difference: oracle {worst_o:.3g}, forward mode {worst_f:.3g}")


def test_adjoint_on_the_greeks_book_fd_options_matches_oracle():
    with open(GOLDEN) as f:
        cases = json.load(f)["greeks_fd32"]
    b = W.book([c["params"] for c in cases])
    say(f"case: reverse-mode Greeks of the 32 FD options of the Greeks book (N {b['N'].min()}..{b['N'].max()})")
    res, g = adjoint(b)
    worst = 0.0
    for i, c in enumerate(cases):
        o = c["oracle"]
        assert res[i]["status"] == 0, (i, res[i]["status"])
        for key in ("ask", "bid", "price0"):
            assert abs(res[i][key] - o[key]) <= 1e-10 * max(abs(o[key]), 1e-300), (i, key)
        for key in ("bp_total_ask", "bp_total_bid", "bp_max_ask", "bp_max_bid"):
            assert int(res[i][key]) == o[key], (i, key)
        for side in ("ask", "bid"):
            e = _rel(grads_of(g[i], side), np.array(o["grad_" + side]))
            worst = max(worst, e)
            assert e <= 1e-9, (i, side)
    say(f"  worst Greek difference {worst:.3g}")


def test_adjoint_against_central_differences():
    book = W.greeks_book(1024, seed=4)
    idx = list(W.greeks_fd_subset(len(book))[:12])
    say("case: reverse-mode Greeks vs central differences, 12 options of the Greeks book")
    passed, kinked, failed = _fd_check(book, idx, greeks=adjoint)
    say(f"  passed {passed}, passed one-sided at a kink {kinked}, failed {failed}")
    assert failed == 0
    assert passed >= 0.9 * (passed + kinked + failed)


def test_autograd_function_in_adjoint_mode():
    # the torch.autograd.Function over the reverse sweep: prices are the
    # batch entry point's bits, gradients contract bt_price_adjoint_batch's
    # Greeks with the incoming gradients, and agree with forward mode
    import torch
    from paper_1110_2477_amd.autograd import bt_autograd
    b = W.random_small(24, seed=93, n_max=120)
    say(f"case: autograd Function, adjoint mode, {len(b)} options")
    ts = {name: torch.tensor(b[name], dtype=torch.float64, device="cuda", requires_grad=True)
          for name in ("S0", "sigma", "R", "k")}
    ask, bid = bt_autograd(ts["S0"], ts["sigma"], ts["R"], ts["k"], b, mode="adjoint")
    (ask.sum() - 3.0 * bid.sum()).backward()
    res, g = adjoint(b)
    assert np.array_equal(ask.detach().cpu().numpy(), res["ask"])
    assert np.array_equal(bid.detach().cpu().numpy(), res["bid"])
    for name, gname in (("S0", "dS0"), ("sigma", "dsigma"), ("R", "dR"), ("k", "dk")):
        want = g["ask_" + gname] - 3.0 * g["bid_" + gname]
        assert np.array_equal(ts[name].grad.cpu().numpy(), want), name
    fwd = {name: torch.tensor(b[name], dtype=torch.float64, device="cuda", requires_grad=True)
           for name in ("S0", "sigma", "R", "k")}
    fa, fb = bt_autograd(fwd["S0"], fwd["sigma"], fwd["R"], fwd["k"], b, mode="forward")
    (fa.sum() - 3.0 * fb.sum()).backward()
    for name in ts:
        a_, f_ = ts[name].grad.cpu().numpy(), fwd[name].grad.cpu().numpy()
        assert np.max(np.abs(a_ - f_) / np.maximum(1.0, np.abs(f_))) < 1e-9, name
    with pytest.raises(ValueError):
        bt_autograd(ts["S0"], ts["sigma"], ts["R"], ts["k"], b, mode="sideways")
