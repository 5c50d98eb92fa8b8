"""Pins of the oracle's payoff shapes beyond the paper's put, call and bull
spread (no GPU).  Section 3 admits any payoff process (xi, zeta): the holder
who exercises receives xi in cash and zeta shares, settled by delivery or in
cash.  For cash-settled puts and calls, bear spreads and straddles:
  * the ask is the seller's superhedging LP and the bid the best over the
    buyer's stopping times of an LP (the definitions of the two prices);
  * at k = 0, ask = bid = the CRR price, and a cash-settled put or call has
    the delivered one's prices (only xi + zeta S matters without costs);
  * European identities that hold exactly on the tree at k = 0: bull plus
    bear spread pays K2 - K at N, and a straddle is a cash put plus a cash
    call;
  * with costs, settlement matters: the delivered put's seller must also
    cover the cost of the share, so cash and delivery differ;
  * the exact-rational recursion pins the prices, and the breakpoint counts
    up to rounding artefacts of the cash-settled payoffs' kinks."""
import pytest

import oracle
from oracle import definitions as D
from oracle import exact as E

NEW = [oracle.PUT_CASH, oracle.CALL_CASH, oracle.BEAR, oracle.STRADDLE]
CASES = [
    # (payoff, K, K2, k, sigma, R, T)
    (oracle.PUT_CASH, 100.0, 0.0, 0.01, 0.3, 0.05, 1.0),
    (oracle.PUT_CASH, 110.0, 0.0, 0.03, 0.2, 0.08, 0.5),
    (oracle.CALL_CASH, 100.0, 0.0, 0.02, 0.3, 0.05, 1.0),
    (oracle.CALL_CASH, 90.0, 0.0, 0.005, 0.4, 0.02, 2.0),
    (oracle.BEAR, 95.0, 105.0, 0.01, 0.2, 0.1, 0.25),
    (oracle.BEAR, 90.0, 120.0, 0.04, 0.35, 0.03, 1.0),
    (oracle.STRADDLE, 100.0, 0.0, 0.02, 0.3, 0.05, 1.0),
    (oracle.STRADDLE, 95.0, 0.0, 0.005, 0.25, 0.0, 0.5),
]


def _price(case, N, **kw):
    pay, K, K2, k, sig, R, T = case
    return oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, **kw)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("N", [1, 3, 6])
def test_ask_equals_superhedging_lp(case, N):
    pay, K, K2, k, sig, R, T = case
    lp = D.ask_lp(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2)
    assert _price(case, N, sides=1)["ask"] == pytest.approx(lp, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("N", [1, 2, 3])
def test_bid_equals_stopping_time_enumeration(case, N):
    pay, K, K2, k, sig, R, T = case
    b = D.bid_enum(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2)
    assert _price(case, N, sides=2)["bid"] == pytest.approx(b, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("case", [CASES[1], CASES[5], CASES[6]])
@pytest.mark.parametrize("flags", [oracle.EUROPEAN, oracle.COST_AT_T0])
def test_variant_flags_against_their_definitions(case, flags):
    pay, K, K2, k, sig, R, T = case
    lp = D.ask_lp(100.0, K, R, sig, T, k, 4, payoff=pay, K2=K2, flags=flags)
    b = D.bid_enum(100.0, K, R, sig, T, k, 3, payoff=pay, K2=K2, flags=flags)
    assert _price(case, 4, flags=flags, sides=1)["ask"] == pytest.approx(lp, rel=1e-10, abs=1e-10)
    assert _price(case, 3, flags=flags, sides=2)["bid"] == pytest.approx(b, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("pay", NEW)
def test_zero_cost_ask_equals_bid_equals_crr(pay):
    K2 = 120.0 if pay == oracle.BEAR else 0.0
    for N in (10, 200):
        r = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, N, payoff=pay, K2=K2)
        assert r["ask"] == pytest.approx(r["price0"], rel=1e-12, abs=1e-12)
        assert r["bid"] == pytest.approx(r["price0"], rel=1e-12, abs=1e-12)


def test_settlement_matters_only_with_costs():
    for phys, cash in ((oracle.PUT, oracle.PUT_CASH), (oracle.CALL, oracle.CALL_CASH)):
        a0 = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, 150, payoff=phys)
        b0 = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, 150, payoff=cash)
        for key in ("ask", "bid", "price0"):
            assert a0[key] == pytest.approx(b0[key], rel=1e-12)
        a1 = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.01, 150, payoff=phys)
        b1 = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.01, 150, payoff=cash)
        assert a1["price0"] == b1["price0"]
        assert abs(a1["ask"] - b1["ask"]) > 1e-3
        # the trivial bounds still hold for both
        for r in (a1, b1):
            assert r["bid"] <= r["price0"] + 1e-12 <= r["ask"] + 2e-12


def test_european_identities_on_the_tree():
    R, T, N = 0.05, 1.0, 120
    eu = oracle.EUROPEAN
    bull = oracle.price(100.0, 95.0, R, 0.3, T, 0.0, N, payoff=oracle.BULL, K2=110.0, flags=eu)
    bear = oracle.price(100.0, 95.0, R, 0.3, T, 0.0, N, payoff=oracle.BEAR, K2=110.0, flags=eu)
    _, c = oracle.model_table(100.0, 0.3, R, T, N)
    assert bull["price0"] + bear["price0"] == pytest.approx(15.0 * c["rho"] ** N, rel=1e-12)
    assert bull["ask"] + bear["ask"] == pytest.approx(15.0 * c["rho"] ** N, rel=1e-12)
    st = oracle.price(100.0, 100.0, R, 0.3, T, 0.0, N, payoff=oracle.STRADDLE, flags=eu)
    pc = oracle.price(100.0, 100.0, R, 0.3, T, 0.0, N, payoff=oracle.PUT_CASH, flags=eu)
    cc = oracle.price(100.0, 100.0, R, 0.3, T, 0.0, N, payoff=oracle.CALL_CASH, flags=eu)
    for key in ("price0", "ask", "bid"):
        assert st[key] == pytest.approx(pc[key] + cc[key], rel=1e-12)


@pytest.mark.parametrize("case", [(oracle.PUT_CASH, 100.0, 0.0, 0.06, 0.3, 0.05, 1.0, 20, 0),
                                  (oracle.CALL_CASH, 100.0, 0.0, 0.08, 0.3, 0.05, 1.0, 16, 0),
                                  (oracle.BEAR, 90.0, 110.0, 0.06, 0.3, 0.05, 1.0, 20, 0),
                                  (oracle.STRADDLE, 100.0, 0.0, 0.05, 0.3, 0.05, 1.0, 16, 0)])
def test_exact_rational_recursion(case):
    pay, K, K2, k, sig, R, T, N, flags = case
    tab, c = oracle.model_table(100.0, sig, R, T, N)
    ex = E.price(tab, c["rho"], k, N, pay, K, K2, flags=flags)
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags)
    for side in ("ask", "bid"):
        ref = float(ex[side])
        assert abs(o[side] - ref) <= 1e-12 * max(1.0, abs(ref)), (side, o[side], ref)
        # with a cash-settled payoff rounding moves kinks both ways: pieces
        # whose exact slopes agree can stay split in binary64, and a crossing
        # that lies just inside an interval exactly can round onto its end
        # (no new point); the counts agree within 5 % (and 2 on the maximum)
        te, tb = ex["kinks_total_" + side], o["bp_total_" + side]
        assert abs(te - tb) <= 0.05 * te, (side, te, tb)
        assert abs(ex["kinks_max_" + side] - o["bp_max_" + side]) <= 2


def test_invalid_spreads_are_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.01, 10, payoff=oracle.BEAR, K2=90.0)
    with pytest.raises(oracle.OracleError):
        oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.01, 10, payoff=7)
