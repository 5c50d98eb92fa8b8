"""Greeks through the C ABI (and the autograd.Function) against the oracle's
forward-mode derivatives and against finite differences of the GPU prices.
Pass rule for finite differences: |AD - FD| <= 1e-6 max(1, |FD|), with the
step refined where the bracket straddles a kink of the piecewise-smooth
price."""
import sys

import numpy as np
import pytest

import oracle
import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

pytestmark = pytest.mark.gpu
KEYS = ("S0", "sigma", "R", "k")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    bt.lib()
    yield


def grads_of(g, side):
    return np.array([g[f"{side}_d{k}"] for k in ("S0", "sigma", "R", "k")])


def test_greeks_match_oracle_tangents():
    b = W.random_small(80, seed=17, n_max=200)
    say("case: Greeks of 80 random options vs oracle tangents")
    res, g = bt.price_book_grad(b)
    plain = bt.price_book(b)
    worst = 0.0
    for i in range(len(b)):
        o = oracle.price_params(b[i], grad=True)
        assert res[i]["status"] == 0
        assert res[i]["ask"] == plain[i]["ask"] and res[i]["bid"] == plain[i]["bid"]
        assert res[i]["ask"] == o["ask"] and res[i]["bid"] == o["bid"]
        for side in ("ask", "bid"):
            ad = grads_of(g[i], side)
            ref = o["grad_" + side]
            err = np.max(np.abs(ad - ref) / np.maximum(1.0, np.abs(ref)))
            worst = max(worst, err)
            assert err <= 1e-9, (i, side, ad, ref)
    say(f"  worst relative difference {worst:.3g}")


def test_greeks_of_invalid_option_are_nan():
    b = W.book([dict(S0=100.0, K=100.0, R=0.05, sigma=0.2, T=1.0, k=0.005, N=40, payoff=W.PUT),
                dict(S0=100.0, K=100.0, R=0.05, sigma=0.2, T=1.0, k=2.0, N=40, payoff=W.PUT)])
    res, g = bt.price_book_grad(b)
    assert res[1]["status"] == bt.BT_EINVAL
    assert all(np.isnan(g[1][n]) for n in g.dtype.names)
    assert all(np.isfinite(g[0][n]) for n in g.dtype.names)


TOL = 1e-6


def _close(x, y):
    return abs(x - y) <= TOL * max(1.0, abs(y))


def _step(p, key, h_rel):
    # relative to S0; absolute for sigma, R and k (rates and cost ratios of
    # order 0.001 - 0.1 would otherwise get steps below the rounding noise of
    # an N-level recursion, about 1e-13 of the price)
    return h_rel * abs(p[key]) if key == "S0" else h_rel


def _fd_check(book, idx, h_rels=(1e-5, 1e-6, 1e-7, 1e-8), greeks=None):
    """Finite differences of GPU prices against the Greeks of the same GPU.

    A binomial price is piecewise smooth in every parameter (a node switching
    between exercise and continuation, or a breakpoint crossing a grid
    price, makes a kink), so a bracket [theta - h, theta + h] may straddle a
    kink.  For each (option, parameter, side) the check runs h = h_rel |theta|
    for decreasing h_rel: it passes as soon as the central difference agrees
    with the derivative; a bracket whose forward and backward one-sided
    differences disagree holds a kink and moves on to a smaller h; at the
    smallest h a kinked bracket passes if the derivative equals one of the
    one-sided slopes (the branch active at theta).  ``greeks`` (default:
    a Greeks book) maps a parameter array to its (results, Greeks).  Returns
    (passed, kink_passed, failed)."""
    base_res, base_g = (greeks or bt.price_book_grad)(book[idx])
    todo = [(j, n, side) for j in range(len(idx)) for n in range(len(KEYS)) for side in ("ask", "bid")]
    passed = kinked = failed = 0
    for level, h_rel in enumerate(h_rels):
        lastlevel = level == len(h_rels) - 1
        rows_p, rows_m, hp, hm = [], [], [], []
        for j, i in enumerate(idx):
            for key in KEYS:
                p = book[i].copy()
                h = _step(p, key, h_rel)
                pp, pm = p.copy(), p.copy()
                pp[key] += h
                pm[key] -= h
                hm_ = h
                if key == "k" and pm[key] < 0:   # one-sided at k = 0
                    pm = p.copy()
                    hm_ = 0.0
                rows_p.append(pp)
                rows_m.append(pm)
                hp.append(h)
                hm.append(hm_)
        rp = bt.price_book(np.array(rows_p))
        rm = bt.price_book(np.array(rows_m))
        assert np.all(rp["status"] == 0) and np.all(rm["status"] == 0)
        nxt = []
        for j, n, side in todo:
            q = j * len(KEYS) + n
            f0 = base_res[j][side]
            ad = grads_of(base_g[j], side)[n]
            fwd = (rp[q][side] - f0) / hp[q]
            if hm[q] == 0.0:
                cen, bwd = fwd, fwd
            else:
                cen = (rp[q][side] - rm[q][side]) / (hp[q] + hm[q])
                bwd = (f0 - rm[q][side]) / hm[q]
            if _close(ad, cen):
                passed += 1
            elif not lastlevel:
                nxt.append((j, n, side))
            elif not _close(fwd, bwd) and (_close(ad, fwd) or _close(ad, bwd)):
                kinked += 1
            else:
                failed += 1
                say(f"  FD failure option {idx[j]} {side} d/d{KEYS[n]}: AD {ad} central {cen} "
                    f"fwd {fwd} bwd {bwd}")
        todo = nxt
        if not todo:
            break
    return passed, kinked, failed


def test_greeks_book_fd_on_32_options():
    # mixed book with N in [500, 1500] (the Greeks workload), 32 options
    book = W.greeks_book(1024, seed=4)
    idx = list(np.random.Generator(np.random.PCG64(44)).choice(len(book), 32, replace=False))
    say("case: Greeks book, FD check on 32 options")
    passed, kinked, failed = _fd_check(book, idx)
    say(f"  passed {passed}, passed one-sided at a kink {kinked}, failed {failed}")
    assert failed == 0
    assert passed >= 0.9 * (passed + kinked + failed)


def test_autograd_function_backward():
    import torch
    from paper_1110_2477_amd.autograd import bt_autograd
    b = W.random_small(6, seed=5, n_max=120)
    S0 = torch.tensor(b["S0"], dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(b["sigma"], dtype=torch.float64, requires_grad=True)
    R = torch.tensor(b["R"], dtype=torch.float64, requires_grad=True)
    k = torch.tensor(b["k"], dtype=torch.float64, requires_grad=True)
    ask, bid = bt_autograd(S0, sig, R, k, b)
    (2.0 * ask.sum() - 3.0 * bid.sum()).backward()
    for i in range(len(b)):
        o = oracle.price_params(b[i], grad=True)
        want = 2.0 * o["grad_ask"] - 3.0 * o["grad_bid"]
        got = np.array([S0.grad[i].item(), sig.grad[i].item(), R.grad[i].item(), k.grad[i].item()])
        assert np.allclose(got, want, rtol=1e-9, atol=1e-9), (i, got, want)


def test_stress_book_sample_graph_greeks_vs_oracle():
    """The stress mix (N log-uniform in [64, 8192], k up to 2 %, puts, calls
    and bull spreads): a seeded sample of its options small enough for the
    oracle, priced with Greeks through a captured HIP graph with 16-level
    bands, against the oracle's values and tangents."""
    s = W.stress_book(16384, seed=5)
    small = np.flatnonzero(s["N"] <= 160)
    pick = np.sort(np.random.Generator(np.random.PCG64(55)).choice(small, 48, replace=False))
    b = s[pick]
    say(f"case: stress-book sample, {len(b)} options with N <= 160, graph + Greeks, band 16")
    bk = bt.Book(b, tune=dict(band_levels=16), greeks=True, graph=True)
    bk.price_grad()
    assert bk.resolve_overflow(grad=True) == 0
    res, g = bk.results(), bk.grads()
    bk.price_grad()   # a replay gives the same bytes
    assert bk.results().tobytes() == res.tobytes() and bk.grads().tobytes() == g.tobytes()
    bk.close()
    for i in range(len(b)):
        o = oracle.price_params(b[i], grad=True)
        assert res[i]["status"] == 0
        assert res[i]["ask"] == o["ask"] and res[i]["bid"] == o["bid"] and res[i]["price0"] == o["price0"], i
        assert res[i]["bp_total_ask"] == o["bp_total_ask"] and res[i]["bp_total_bid"] == o["bp_total_bid"], i
        for side in ("ask", "bid"):
            ad = grads_of(g[i], side)
            ref = o["grad_" + side]
            err = np.max(np.abs(ad - ref) / np.maximum(1.0, np.abs(ref)))
            assert err <= 1e-9, (i, side, ad, ref)
