"""Pins of the C oracle against the exact-rational recursion (no GPU).

``oracle/exact.py`` runs Section 3's recursions in exact rational arithmetic
from the same binary64 inputs (stock table, rho, and the node constants
a = -(1+k)S, b = -(1-k)S, xi, zeta), written from the definitions of the
maximum, the discount, the restriction (an inf-convolution with the cost
cone) and the exercise step, with none of the C oracle's operation orders or
tie rules.  It pins
  * the prices: the binary64 recursion may differ only by its rounding;
  * the breakpoint counts: every genuine kink of the exact functions must
    show in the binary64 counts, and for puts and calls (whose expense
    functions have no cash-settled payoff kinks) the counts must be equal.
    A cash-settled bull spread can leave binary64 kinks between pieces
    whose exact slopes agree (rounding artefacts), so there the binary64
    count may only be larger.
"""
import pytest

import oracle
from oracle import exact as E

# (payoff, K, K2, k, sigma, R, T, N, flags)
CASES = [
    (oracle.PUT, 100.0, 0.0, 0.1, 0.3, 0.05, 1.0, 24, 0),
    (oracle.PUT, 110.0, 0.0, 0.06, 0.25, 0.08, 0.5, 30, 0),
    (oracle.CALL, 100.0, 0.0, 0.06, 0.3, 0.05, 1.0, 24, 0),
    (oracle.CALL, 90.0, 0.0, 0.1, 0.3, 0.05, 1.0, 20, 0),
    (oracle.CALL, 100.0, 0.0, 0.1, 0.3, 0.05, 1.0, 12, 0),
    (oracle.BULL, 95.0, 110.0, 0.06, 0.3, 0.05, 1.0, 24, 0),
    (oracle.BULL, 100.0, 125.0, 0.1, 0.3, 0.05, 1.0, 24, 0),
    (oracle.CALL, 100.0, 0.0, 0.08, 0.3, 0.05, 1.0, 16, oracle.EUROPEAN),
    (oracle.PUT, 100.0, 0.0, 0.05, 0.3, 0.05, 1.0, 16, oracle.COST_AT_T0),
    (oracle.BULL, 95.0, 105.0, 0.01, 0.2, 0.1, 0.25, 30, 0),
]


@pytest.mark.parametrize("case", CASES)
def test_exact_rational_recursion_pins_prices_and_kinks(case):
    pay, K, K2, k, sig, R, T, N, flags = case
    tab, c = oracle.model_table(100.0, sig, R, T, N)
    ex = E.price(tab, c["rho"], k, N, pay, K, K2, flags=flags)
    o = oracle.price(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags)
    for side in ("ask", "bid"):
        ref = float(ex[side])
        assert abs(o[side] - ref) <= 1e-12 * max(1.0, abs(ref)), (side, o[side], ref)
        tot, mx = ex["kinks_total_" + side], ex["kinks_max_" + side]
        assert tot <= o["bp_total_" + side] and mx <= o["bp_max_" + side], (side, tot, mx)
        if pay != oracle.BULL:
            assert (tot, mx) == (o["bp_total_" + side], o["bp_max_" + side]), side


def test_exact_counts_see_growth():
    # the cases above are only a pin on the counts if breakpoints grow: the
    # high-cost call's buyer reaches many kinks per node (2k / (sigma
    # sqrt(T/N)) > 1 keeps the children's middle pieces)
    tab, c = oracle.model_table(100.0, 0.3, 0.05, 1.0, 20)
    ex = E.price(tab, c["rho"], 0.1, 20, oracle.CALL, 90.0)
    assert ex["kinks_max_bid"] >= 10


def test_exact_envelope_and_restriction_definitions():
    # the exact operations against hand-computed functions
    from fractions import Fraction as F
    f = E.Pwl([F(0)], [F(0)], [F(-3), F(1)])            # slopes -3 / 1, kink at 0
    g = E.Pwl([F(1)], [F(-1)], [F(-1), F(-1)])          # the line -y
    # y < 0: -3y > -y; y > 0: y > -y; so max is f and min is -y
    m = E.envelope([f, g], max)
    assert m.xs == [F(0)] and m.ss == [F(-3), F(1)]
    n = E.envelope([f, g], min)
    assert n.kinks() == 0 and n(F(2)) == F(-2) and n(F(-5)) == F(5)
    # restriction of a convex function: its slopes clamped into [a, b]
    r = E.restrict(f, F(-2), F(-1, 2))
    assert r.ss == [F(-2), F(-1, 2)] and r(F(0)) == 0
    # a non-convex function against the inf-convolution written out: a
    # holding y can be moved to y' at cost (-a)(y' - y) when buying and
    # b (y - y') when selling (a < b < 0)
    w = E.Pwl([F(-1), F(0), F(1)], [F(0), F(1), F(0)], [F(-4), F(1), F(-1), F(4)])
    a, b = F(-3, 2), F(-1, 2)
    rw = E.restrict(w, a, b)
    for y in [F(q, 4) for q in range(-12, 13)]:
        cands = [w(y)] + [w(x) + ((-a) * (x - y) if x >= y else b * (y - x)) for x in w.xs]
        assert rw(y) == min(cands), y
    assert all(a <= s <= b for s in rw.ss)
