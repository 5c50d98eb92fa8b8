"""Pins of the oracle's hedging output: the optimal stock holding at t = 0
of the seller and of the buyer (no GPU).

From the epigraph reading of Section 3, the root's restriction is
v_0(0) = min over y of f(y) + (cost of buying y shares at t = 0), with
f = rho max(z_1(1), z_1(0)); the minimisers are the holdings the hedger
carries to t = 1.  Pinned by:
  * the superhedging LP: its optimal portfolio's holding after t = 0 lies in
    the seller's interval whenever continuation beats immediate exercise;
  * k = 0: the seller holds the CRR delta (V_1(1) - V_1(0)) / (S_1(1) -
    S_1(0)), and the buyer the opposite position."""
import pytest

import oracle
from oracle import definitions as D

CASES = [
    # (payoff, K, K2, k, sigma, R, T)
    (oracle.PUT, 100.0, 0.0, 0.01, 0.3, 0.05, 1.0),
    (oracle.PUT, 90.0, 0.0, 0.03, 0.2, 0.08, 0.5),
    (oracle.CALL, 100.0, 0.0, 0.02, 0.3, 0.05, 1.0),
    (oracle.CALL_CASH, 95.0, 0.0, 0.005, 0.4, 0.02, 2.0),
    (oracle.BULL, 95.0, 105.0, 0.01, 0.2, 0.1, 0.25),
    (oracle.STRADDLE, 100.0, 0.0, 0.02, 0.3, 0.05, 1.0),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("N", [2, 4, 6])
def test_seller_hedge_holds_the_lp_portfolio(case, N):
    pay, K, K2, k, sig, R, T = case
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, sides=1)
    h = oracle.hedge(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2)["ask"]
    xi, ze = D._payoff(pay, 100.0, K, K2)
    exercise_now = xi + ze * 100.0   # the seller's u_0(0) with no cost at t = 0
    if o["ask"] <= exercise_now + 1e-9:
        pytest.skip("immediate exercise binds: every holding that covers it is optimal")
    val, y = D.ask_lp(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, with_hedge=True)
    assert val == pytest.approx(o["ask"], rel=1e-10, abs=1e-10)
    assert h[0] - 1e-7 <= y <= h[1] + 1e-7, (h, y)


@pytest.mark.parametrize("pay", [oracle.PUT, oracle.CALL, oracle.PUT_CASH, oracle.BULL, oracle.STRADDLE])
@pytest.mark.parametrize("N", [3, 50, 400])
def test_zero_cost_hedge_is_the_crr_delta(pay, N):
    K2 = 115.0 if pay == oracle.BULL else 0.0
    V, S = D.crr_values(100.0, 100.0, 0.05, 0.3, 1.0, N, payoff=pay, K2=K2, level=1)
    delta = (V[1] - V[0]) / (S[1] - S[0])
    h = oracle.hedge(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, N, payoff=pay, K2=K2)
    assert h["ask"][0] == pytest.approx(delta, rel=1e-9, abs=1e-11)
    assert h["ask"][1] == pytest.approx(delta, rel=1e-9, abs=1e-11)
    assert h["bid"][0] == pytest.approx(-delta, rel=1e-9, abs=1e-11)
    assert h["bid"][1] == pytest.approx(-delta, rel=1e-9, abs=1e-11)


def test_costs_widen_what_the_two_parties_hold():
    # with costs the seller of a put shorts fewer shares than the zero-cost
    # delta or keeps the same, and the two parties no longer hold opposite
    # positions
    h0 = oracle.hedge(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, 200)
    h1 = oracle.hedge(100.0, 100.0, 0.05, 0.3, 1.0, 0.01, 200)
    assert h1["ask"][0] != h0["ask"][0]
    assert h1["ask"][0] != -h1["bid"][0]
