"""Pins of the oracle's forward-mode Greeks against central finite differences
of its own prices (no GPU).  Pass rule: |AD - FD| <= 1e-6 max(1, |FD|), the
Greeks tolerance for this path; the bumps stay on one side of every kink for
these cases (checked by comparing the breakpoint counts at +h and -h)."""
import pytest

import oracle

KEYS = ["S0", "sigma", "R", "k"]
CASES = [
    (oracle.PUT, 100.0, 0.005, 50),
    (oracle.CALL, 100.0, 0.01, 80),
    (oracle.BULL, 95.0, 0.01, 60),
    (oracle.PUT, 110.0, 0.02, 100),
    (oracle.CALL, 90.0, 0.003, 150),
]


@pytest.mark.parametrize("case", CASES)
def test_tangents_match_central_differences(case):
    pay, K, k, N = case
    p = dict(S0=100.0, K=K, K2=105.0, R=0.05, sigma=0.3, T=1.0, k=k, N=N, payoff=pay, flags=0)
    g = oracle.price_params(p, grad=True)
    base = oracle.price_params(p)
    # values of the tangent build equal those of the value-only build
    for key in ("ask", "bid", "price0", "bp_total_ask", "bp_total_bid"):
        assert g[key] == base[key]
    for i, key in enumerate(KEYS):
        h = 1e-5 * max(abs(p[key]), 1e-3)
        pp, pm = dict(p), dict(p)
        pp[key] += h
        pm[key] -= h
        rp, rm = oracle.price_params(pp), oracle.price_params(pm)
        for side in ("ask", "bid"):
            fd = (rp[side] - rm[side]) / (2 * h)
            ad = g["grad_" + side][i]
            assert abs(ad - fd) <= 1e-6 * max(1.0, abs(fd)), (side, key, ad, fd)


def test_delta_of_deep_put_bid_is_minus_one():
    # K = 110, k = 2%: the buyer exercises at once (bid = K - S0), so the bid's
    # delta is exactly -1 and its other Greeks vanish.
    g = oracle.price(100.0, 110.0, 0.05, 0.3, 1.0, 0.02, 100, grad=True)
    assert g["bid"] == pytest.approx(10.0, abs=1e-12)
    assert g["grad_bid"][0] == -1.0
    assert list(g["grad_bid"][1:]) == [0.0, 0.0, 0.0] or all(abs(x) == 0.0 for x in g["grad_bid"][1:])
