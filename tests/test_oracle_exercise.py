"""Pins of the oracle's exercise maps (no GPU).

The exercise map of a party marks the nodes at which exercise attains the
party's expense at zero stock holding (Section 3: the seller's z_t is the
larger of the exercise expense u_t and the continuation v_t, the buyer's the
smaller).  The oracle decides it from its own binary64 functions as
EVAL(u_t, 0) against EVAL(v_t, 0).  Three things it has to agree with:

  * the exact-rational recursion's u_t(0) against v_t(0) (written from the
    definitions, with none of the oracle's operation orders), on every node
    whose two exact values are not within rounding of each other;
  * at k = 0 the classic zero-cost stopping region {xi + zeta S >=
    continuation} of the scalar recursion, for both parties;
  * the European variant: no exercise before N.
"""
import numpy as np
import pytest

import oracle
from oracle import definitions as D
from oracle import exact as E

# (payoff, K, K2, k, sigma, R, T, N, flags)
CASES = [
    (oracle.PUT, 100.0, 0.0, 0.05, 0.3, 0.05, 1.0, 14, 0),
    (oracle.PUT, 110.0, 0.0, 0.02, 0.25, 0.08, 0.5, 16, 0),
    (oracle.CALL, 100.0, 0.0, 0.04, 0.3, 0.05, 1.0, 12, 0),
    (oracle.BULL, 95.0, 110.0, 0.03, 0.3, 0.05, 1.0, 12, 0),
    (oracle.PUT_CASH, 105.0, 0.0, 0.03, 0.3, 0.06, 1.0, 12, 0),
    (oracle.STRADDLE, 100.0, 0.0, 0.02, 0.3, 0.05, 1.0, 10, 0),
    (oracle.PUT, 100.0, 0.0, 0.05, 0.3, 0.05, 1.0, 10, oracle.COST_AT_T0),
    (oracle.CALL, 100.0, 0.0, 0.05, 0.3, 0.05, 1.0, 10, oracle.EUROPEAN),
]


def _node(t, c):
    return t * (t + 1) // 2 + c


@pytest.mark.parametrize("case", CASES)
def test_exercise_map_matches_exact_recursion(case):
    pay, K, K2, k, sig, R, T, N, flags = case
    tab, cst = oracle.model_table(100.0, sig, R, T, N)
    from fractions import Fraction as F
    ftab = [F(float(s)) for s in tab]
    m = oracle.exercise(100.0, K, R, sig, T, k, N, payoff=pay, K2=K2, flags=flags)
    decided = allowed = 0
    for side in (0, 1):
        ex = {}
        E.side_price(lambda j: ftab[j + N + 1], F(float(cst["rho"])), F(float(k)), N, pay, F(K), F(K2), side,
                     flags, True, exmap=ex)
        for t in range(N + 1):
            for c in range(t + 1):
                got = int(m[side, _node(t, c)])
                if (t, c) not in ex:
                    assert got == 0, (side, t, c)
                    continue
                u0, v0 = ex[(t, c)]
                allowed += 1
                scale = max(1.0, abs(float(u0)), abs(float(v0)))
                if abs(float(u0 - v0)) <= 1e-9 * scale:
                    continue   # within rounding of a tie: either answer
                want = int(u0 > v0) if side == 0 else int(u0 < v0)
                assert got == want, (side, t, c, float(u0), float(v0))
                decided += 1
    # the comparison decided most nodes (the pin is not vacuous)
    assert decided >= 0.6 * allowed


@pytest.mark.parametrize("pay,K,K2", [(oracle.PUT, 100.0, 0.0), (oracle.PUT, 120.0, 0.0), (oracle.CALL, 95.0, 0.0),
                                      (oracle.PUT_CASH, 100.0, 0.0), (oracle.BEAR, 95.0, 110.0)])
def test_exercise_map_at_zero_cost_is_the_crr_stopping_region(pay, K, K2):
    N, sig, R, T = 60, 0.3, 0.06, 1.0
    m = oracle.exercise(100.0, K, R, sig, T, 0.0, N, payoff=pay, K2=K2)
    flg, mrg = D.crr_exercise(100.0, K, R, sig, T, N, payoff=pay, K2=K2)
    clear = np.abs(mrg) > 1e-9 * np.maximum(1.0, np.abs(mrg + 0.0))
    for side in (0, 1):
        bad = np.nonzero(clear & (m[side] != flg))[0]
        assert bad.size == 0, (side, bad[:5])
    # both exercise and continuation occur (a put deep in the money is
    # exercised early, out of the money never)
    assert 0 < flg.sum() < flg.size


def test_exercise_map_european_has_no_early_exercise():
    N = 40
    m = oracle.exercise(100.0, 100.0, 0.05, 0.3, 1.0, 0.01, N, payoff=oracle.PUT, flags=oracle.EUROPEAN)
    assert not m[:, :_node(N, 0)].any()
    # at N the put is exercised in the money
    last = m[:, _node(N, 0):]
    assert last.any()


def test_exercise_map_put_region_shape():
    # an American put with costs: the seller's continuation expense at zero
    # holding is never negative (the holder may never exercise), so the
    # seller's exercise nodes have K - (1 - k_t) S >= 0; and deep in the
    # money the buyer exercises at the last level
    N, K, k = 80, 100.0, 0.005
    m = oracle.exercise(100.0, K, 0.06, 0.3, 1.0, k, N, payoff=oracle.PUT)
    tab, _ = oracle.model_table(100.0, 0.3, 0.06, 1.0, N)
    for t in range(N + 1):
        kt = k if t >= 1 else 0.0
        for c in range(t + 1):
            S = tab[2 * c - t + N + 1]
            if m[0, _node(t, c)]:
                assert K - (1.0 - kt) * S >= 0.0, (t, c, S)
    assert m[1, _node(N, 0)] == 1
