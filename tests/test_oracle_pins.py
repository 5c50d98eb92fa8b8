"""Pins of the CPU oracle against what the paper and the mathematics fix
(no GPU).  Each test names the passage or fact it rests on."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import definitions as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# P1: the worked one-step example of Section 3.
# ---------------------------------------------------------------------------
def _load_example():
    with open(os.path.join(GOLDEN, "one_step_example.json")) as f:
        return json.load(f)


def _vee(kink, value, sl, sr):
    return ([kink], [value], [sl, sr])


def test_worked_example_seller_and_buyer():
    ex = _load_example()
    pr = ex["printed"]
    S, u, k, K, r = ex["S_t"], ex["u"], ex["k"], ex["K"], ex["r"]
    d = 1.0 / u
    # the printed child slopes are (1 +- k) S u and (1 +- k) S d
    Su, Sd = S * u, S * d
    assert (1 + k) * Su == pytest.approx(-pr["seller_child_up"]["slope_left"])
    assert (1 - k) * Sd == pytest.approx(-pr["seller_child_down"]["slope_right"], abs=5e-3)
    zu = _vee(-1.0, K, -(1 + k) * Su, -(1 - k) * Su)
    zd = _vee(-1.0, K, -(1 + k) * Sd, -(1 - k) * Sd)
    z, v = oracle.node(0, zu, zd, S, k, 1.0 / r, K, -1.0)
    # v_t = 110.1695 + 120 (y+1)^- - 80 (y+1)^+ (the discounted, restricted max)
    assert np.allclose(v[0], [-1.0]) and v[1][0] == pytest.approx(K / r, rel=1e-15)
    assert list(v[2]) == [-120.0, -80.0]
    # z_t = u_t, with pieces -120 y + 10 (y < -1) and -80 y + 50 (y >= -1)
    for y in (-3.0, -1.5, -1.0, 0.0, 2.0):
        (sl, ic) = pr["seller_z_t_pieces"][0 if y < pr["seller_z_t_break"] else 1]
        assert oracle.pwl_eval(z, y) == pytest.approx(sl * y + ic, rel=1e-14)
    assert oracle.pwl_eval(z, 0.0) == pr["ask"]
    # buyer: children and u_t with kink at -zeta = 1 and value -xi
    zu = _vee(1.0, -K, -(1 + k) * Su, -(1 - k) * Su)
    zd = _vee(1.0, -K, -(1 + k) * Sd, -(1 - k) * Sd)
    z, v = oracle.node(1, zu, zd, S, k, 1.0 / r, K, -1.0)
    for y in (-2.0, 0.0, 1.0, 3.0):
        (sl, ic) = pr["buyer_z_t_pieces"][0 if y < pr["buyer_z_t_break"] else 1]
        assert oracle.pwl_eval(z, y) == pytest.approx(sl * y + ic, rel=1e-14)
    assert -oracle.pwl_eval(z, 0.0) == pr["bid"]


def test_worked_example_zero_cost_numbers():
    ex = _load_example()
    pr = ex["printed"]
    u, r, S, K = ex["u"], ex["r"], ex["S_t"], ex["K"]
    d = 1.0 / u
    p = (r - d) / (u - d)
    assert abs(p - pr["p"]) < 1e-4
    assert K - S * u == pytest.approx(pr["payoff_up"])
    assert K - S * d == pytest.approx(pr["payoff_down"], abs=5e-3)


# ---------------------------------------------------------------------------
# P5 / P6: the ask is the seller's superhedging LP, the bid the best over the
# buyer's stopping times of an LP (Section 3's definitions of the two prices).
# ---------------------------------------------------------------------------
LP_CASES = [
    # (payoff, K, K2, k, sigma, R, T)
    (oracle.PUT, 100.0, 0.0, 0.01, 0.3, 0.05, 1.0),
    (oracle.PUT, 110.0, 0.0, 0.03, 0.2, 0.08, 0.5),
    (oracle.CALL, 100.0, 0.0, 0.02, 0.3, 0.05, 1.0),
    (oracle.CALL, 90.0, 0.0, 0.005, 0.4, 0.02, 2.0),
    (oracle.BULL, 95.0, 105.0, 0.01, 0.2, 0.1, 0.25),
    (oracle.BULL, 100.0, 120.0, 0.04, 0.35, 0.03, 1.0),
    (oracle.PUT, 100.0, 0.0, 0.0, 0.3, 0.05, 1.0),
]


@pytest.mark.parametrize("case", LP_CASES)
@pytest.mark.parametrize("N", [1, 2, 4, 7, 8])
def test_ask_equals_superhedging_lp(case, N):
    pay, K, K2, k, sig, R, T = case
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, sides=1)
    lp = D.ask_lp(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2)
    assert o["ask"] == pytest.approx(lp, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("case", LP_CASES[:6])
@pytest.mark.parametrize("N", [1, 2])
def test_bid_equals_stopping_time_enumeration(case, N):
    pay, K, K2, k, sig, R, T = case
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, sides=2)
    b = D.bid_enum(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2)
    assert o["bid"] == pytest.approx(b, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("case", [LP_CASES[0], LP_CASES[2], LP_CASES[4]])
def test_bid_equals_stopping_time_enumeration_n3(case):
    pay, K, K2, k, sig, R, T = case
    o = oracle.price(100.0, K, R, sig, T, k, 3, payoff=pay, K2=K2, sides=2)
    b = D.bid_enum(100.0, K, R, sig, T, k, 3, payoff=pay, K2=K2)
    assert o["bid"] == pytest.approx(b, rel=1e-10, abs=1e-10)


# The two variants of the model: costs charged at t = 0 as well (the paper
# charges none there, Section 4.1), and exercise at N only (European).  The
# linear programs change only where the definition does: the cost rate of
# the trades at t = 0, and the times at which delivery must be covered (the
# seller) or the buyer may stop.
VARIANT_CASES = [LP_CASES[0], LP_CASES[2], LP_CASES[4], LP_CASES[5]]


@pytest.mark.parametrize("case", VARIANT_CASES)
@pytest.mark.parametrize("flags", [oracle.COST_AT_T0, oracle.EUROPEAN, oracle.EUROPEAN | oracle.COST_AT_T0])
@pytest.mark.parametrize("N", [2, 5])
def test_variant_ask_equals_superhedging_lp(case, flags, N):
    pay, K, K2, k, sig, R, T = case
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags, sides=1)
    lp = D.ask_lp(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags)
    assert o["ask"] == pytest.approx(lp, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("case", VARIANT_CASES)
@pytest.mark.parametrize("flags", [oracle.COST_AT_T0, oracle.EUROPEAN, oracle.EUROPEAN | oracle.COST_AT_T0])
@pytest.mark.parametrize("N", [2, 3])
def test_variant_bid_equals_stopping_time_enumeration(case, flags, N):
    pay, K, K2, k, sig, R, T = case
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags, sides=2)
    b = D.bid_enum(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags)
    assert o["bid"] == pytest.approx(b, rel=1e-10, abs=1e-10)


def test_variants_change_the_prices():
    # the variant pins above would pass for an oracle that ignored the flags
    # only if the flags did not matter: check that they do
    # (the European variant of a call on a stock without dividends is worth
    # the American call, so the put shows that flag)
    for case, fl in ((LP_CASES[2], oracle.COST_AT_T0), (LP_CASES[0], oracle.EUROPEAN),
                     (LP_CASES[4], oracle.COST_AT_T0), (LP_CASES[4], oracle.EUROPEAN)):
        pay, K, K2, k, sig, R, T = case
        base = oracle.price(100.0, K, R, sig, T, k, 5, payoff=pay, K2=K2)
        v = oracle.price(100.0, K, R, sig, T, k, 5, payoff=pay, K2=K2, flags=fl)
        assert abs(v["ask"] - base["ask"]) > 1e-3 and abs(v["bid"] - base["bid"]) > 1e-3


def _enum_golden():
    with open(os.path.join(GOLDEN, "bid_enumeration_n4.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("i", [0, 1])
def test_bid_equals_stopping_time_enumeration_n4(i):
    # all 458,330 stopping times of the N = 4 path tree, each priced by an LP
    # (tests/golden/make_bid_enumeration_n4.py, oracle.definitions only)
    c = _enum_golden()[i]
    assert c["stopping_times"] == D.count_stopping_times(4)
    o = oracle.price(c["S0"], c["K"], c["R"], c["sigma"], c["T"], c["k"], c["N"], payoff=c["payoff"],
                     K2=c["K2"], sides=2)
    assert o["bid"] == pytest.approx(c["bid_enumeration"], rel=1e-10, abs=1e-10)


@pytest.mark.slow
@pytest.mark.parametrize("i", [0, 1])
def test_bid_enumeration_n4_recomputed(i):
    # recomputes the stored enumeration (minutes on 8 cores)
    c = _enum_golden()[i]
    b = D.bid_enum(c["S0"], c["K"], c["R"], c["sigma"], c["T"], c["k"], c["N"], payoff=c["payoff"], K2=c["K2"],
                   workers=os.cpu_count() or 1)
    assert b == pytest.approx(c["bid_enumeration"], rel=1e-12, abs=1e-12)


def test_stopping_time_counts():
    # one stopping time per choice "exercise here or continue on both branches"
    assert [D.count_stopping_times(n) for n in (2, 3, 4)] == [26, 677, 458330]
    assert len(D._stopping_times(2)) == 26
    # European: stop at N or leave unexercised, per path: 2^(2^N)
    assert [len(D._stopping_times(n, oracle.EUROPEAN)) for n in (1, 2, 3)] == [4, 16, 256]


# ---------------------------------------------------------------------------
# P2 / P3 / P8: zero-cost pins (Section 3, Appendix).
# ---------------------------------------------------------------------------
def test_appendix_price_13_906():
    # Appendix: American put K = S0 = 100, T = 3, sigma = 0.3, R = 0.06; the
    # printed price is 13.906 for N between 5000 and 40000 (3 decimals).
    for N in (10000, 20000):
        r = oracle.price(100.0, 100.0, 0.06, 0.3, 3.0, 0.0, N, sides=0)
        assert round(r["price0"], 3) == 13.906


@pytest.mark.parametrize("pay,K,K2", [(oracle.PUT, 100, 0), (oracle.CALL, 95, 0), (oracle.BULL, 95, 105),
                                      (oracle.PUT, 120, 0)])
@pytest.mark.parametrize("N", [1, 7, 64, 301])
def test_zero_cost_ask_equals_bid_equals_crr(pay, K, K2, N):
    # k = 0 makes the price unique (Fig. 5 discussion: pi^a_{k0} = pi^b_{k0})
    # and equal to the scalar recursion of the Appendix.
    r = oracle.price(100.0, K, 0.05, 0.25, 1.0, 0.0, N, payoff=pay, K2=K2)
    assert r["ask"] == pytest.approx(r["price0"], rel=1e-12, abs=1e-12)
    assert r["bid"] == pytest.approx(r["price0"], rel=1e-12, abs=1e-12)
    assert r["bp_total_ask"] == 0 and r["bp_total_bid"] == 0


def _bs(S, K, R, sig, T, call):
    from scipy.stats import norm
    d1 = (math.log(S / K) + (R + 0.5 * sig * sig) * T) / (sig * math.sqrt(T))
    d2 = d1 - sig * math.sqrt(T)
    if call:
        return S * norm.cdf(d1) - K * math.exp(-R * T) * norm.cdf(d2)
    return K * math.exp(-R * T) * norm.cdf(-d2) - S * norm.cdf(-d1)


@pytest.mark.parametrize("pay", [oracle.PUT, oracle.CALL])
def test_european_zero_cost_converges_to_black_scholes(pay):
    bs = _bs(100.0, 105.0, 0.05, 0.3, 1.0, pay == oracle.CALL)
    errs = []
    for N in (250, 1000, 4000):
        r = oracle.price(100.0, 105.0, 0.05, 0.3, 1.0, 0.0, N, payoff=pay, flags=oracle.EUROPEAN)
        assert r["ask"] == pytest.approx(r["price0"], rel=1e-12)
        errs.append(abs(r["price0"] - bs))
    assert errs[-1] < 2e-3
    assert errs[-1] < errs[0]


@pytest.mark.parametrize("N", [10, 333])
def test_european_put_call_parity(N):
    S0, K, R, T = 100.0, 97.0, 0.04, 1.5
    c = oracle.price(S0, K, R, 0.3, T, 0.0, N, payoff=oracle.CALL, flags=oracle.EUROPEAN)
    p = oracle.price(S0, K, R, 0.3, T, 0.0, N, payoff=oracle.PUT, flags=oracle.EUROPEAN)
    rhs = S0 - K * math.exp(-R * T)
    for key in ("price0", "ask", "bid"):
        assert c[key] - p[key] == pytest.approx(rhs, abs=1e-9)


def test_american_call_equals_european_without_costs():
    # Appendix: without dividends or costs the American call is worth the
    # European call.
    a = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, 500, payoff=oracle.CALL)
    e = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.0, 500, payoff=oracle.CALL, flags=oracle.EUROPEAN)
    assert a["price0"] == pytest.approx(e["price0"], rel=1e-12)
    assert a["ask"] == pytest.approx(e["ask"], rel=1e-12)


# ---------------------------------------------------------------------------
# P4: invariants.
# ---------------------------------------------------------------------------
def test_fig5_ordering_of_ask_and_bid_curves():
    # Fig. 5: put K = 100 (the put of the correctness tests: T = 0.25,
    # sigma = 0.2, R = 0.1), S0 = 90..110, k0 = 0 < k1 = 0.25% < k2 = 0.5%.
    for S0 in (90.0, 95.0, 100.0, 105.0, 110.0):
        r = [oracle.price(S0, 100.0, 0.1, 0.2, 0.25, k, 200) for k in (0.0, 0.0025, 0.005)]
        assert r[2]["bid"] <= r[1]["bid"] + 1e-12
        assert r[1]["bid"] <= r[0]["ask"] + 1e-12
        assert r[0]["ask"] == pytest.approx(r[0]["bid"], rel=1e-12)
        assert r[0]["bid"] < r[1]["ask"] < r[2]["ask"]


@pytest.mark.parametrize("pay,K,K2", [(oracle.PUT, 100, 0), (oracle.CALL, 100, 0), (oracle.BULL, 95, 110)])
def test_spread_monotone_in_k_and_brackets_price0(pay, K, K2):
    prev = None
    for k in (0.0, 0.001, 0.004, 0.01, 0.02, 0.05):
        r = oracle.price(100.0, K, 0.05, 0.3, 1.0, k, 150, payoff=pay, K2=K2)
        assert r["bid"] <= r["price0"] + 1e-12 <= r["ask"] + 2e-12
        if prev is not None:
            assert r["ask"] >= prev["ask"] - 1e-12
            assert r["bid"] <= prev["bid"] + 1e-12
        prev = r


def test_trivial_hedges_and_subhedges():
    rng = np.random.default_rng(11)
    for _ in range(12):
        S0 = 100 * math.exp(0.2 * rng.standard_normal())
        K = S0 * rng.uniform(0.8, 1.2)
        sig, T, R, k = rng.uniform(0.1, 0.6), rng.uniform(0.1, 2), rng.uniform(0, 0.08), rng.uniform(0, 0.03)
        N = int(rng.integers(20, 120))
        p = oracle.price(S0, K, R, sig, T, k, N, payoff=oracle.PUT)
        c = oracle.price(S0, K, R, sig, T, k, N, payoff=oracle.CALL)
        disc = math.exp(-R * T)
        # holding K in cash covers the put; holding one share covers the call
        assert p["ask"] <= K + 1e-9 and c["ask"] <= S0 + 1e-9
        # immediate exercise at t = 0 (no cost at t = 0)
        assert p["bid"] >= max(K - S0, 0) - 1e-9 and c["bid"] >= max(S0 - K, 0) - 1e-9
        # static sub-hedges held to expiry
        assert c["bid"] >= S0 - K * disc - 1e-9
        assert p["bid"] >= K * disc - S0 - 1e-9
        for r in (p, c):
            assert r["bid"] <= r["price0"] + 1e-9 <= r["ask"] + 2e-9


def test_extra_level_reproduces_exercise_or_liquidate_at_N():
    # With d < r < u the discounted, restricted maximum of the two liquidation
    # functions at level N+1 is the liquidation function at level N, so an
    # N-step tree and the same tree seen from one step later agree: the
    # one-step tree's ask/bid equal max/min of immediate payoff and
    # liquidation at t = 0 combined through one rebalancing step.
    r = oracle.price(100.0, 100.0, 0.05, 0.3, 1.0, 0.02, 1, payoff=oracle.PUT)
    lp = D.ask_lp(100.0, 100.0, 0.05, 0.3, 1.0, 0.02, 1, payoff=oracle.PUT)
    assert r["ask"] == pytest.approx(lp, rel=1e-12)


def test_invalid_parameters_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.price(100, 100, 0.05, 0.3, 1.0, 1.0, 10)          # k >= 1
    with pytest.raises(oracle.OracleError):
        oracle.price(100, 100, 5.0, 0.01, 1.0, 0.0, 2)           # r > u: arbitrage
    with pytest.raises(oracle.OracleError):
        oracle.price(100, 100, 0.05, 0.3, 1.0, 0.0, 0)           # N < 1
    with pytest.raises(oracle.OracleError):
        oracle.price(100, 100, 0.05, 0.3, 1.0, 0.0, 10, payoff=oracle.BULL, K2=90)


# glibc's exp rounds these arguments to the other neighbour of e^x; the model
# takes u and r correctly rounded (Section 4.1 defines them as exponentials)
_HARD_EXP_ARGS = ["0x1.a056d88f0ced3p-8", "0x1.88ab8b85f2710p-9", "0x1.983139ccee7acp-7",
                  "0x1.6c15d3740474dp-9"]


def test_model_exponentials_are_correctly_rounded():
    # u = e^(sigma sqrt(T/N)) and r = e^(R T/N) against 60-digit decimal
    # arithmetic: with T = N = 1 the exponents are sigma and R themselves
    from decimal import Context, Decimal
    rng = np.random.default_rng(61)
    xs = [float.fromhex(h) for h in _HARD_EXP_ARGS] + list(rng.uniform(1e-4, 0.6, 400))
    for x in xs:
        ref = float(Decimal(x).exp(Context(prec=60)))
        _, c = oracle.model_table(100.0, x, 0.0, 1.0, 1)
        assert c["u"] == ref, x.hex()
        _, c = oracle.model_table(100.0, 1.0, x, 1.0, 1)
        assert c["r"] == ref, x.hex()
    # the general case: sqrt(T/N) too
    for _ in range(200):
        N = int(rng.integers(1, 20000))
        T, sig, R = rng.uniform(0.05, 3), rng.uniform(0.05, 0.8), rng.uniform(0.0, 0.1)
        dt = T / N
        _, c = oracle.model_table(100.0, sig, R, T, N)
        assert c["u"] == float(Decimal(sig * math.sqrt(dt)).exp(Context(prec=60)))
        assert c["r"] == float(Decimal(R * dt).exp(Context(prec=60)))
        assert c["d"] == 1.0 / c["u"] and c["rho"] == 1.0 / c["r"]
