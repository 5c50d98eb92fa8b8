"""Plain definitions that pin the oracle's recursion (test infrastructure).

The paper (Section 3) defines the ask as the least initial wealth with which
the seller can hedge the option without risk, and the bid as the most the
buyer can borrow against the right to exercise.  On the non-recombining path
tree those are linear programs:

* ``ask_lp``: minimise the seller's initial cash x such that a self-financing
  strategy starting from (x, 0) keeps the portfolio that arrives at every node
  of times 0..N+1 inside the epigraph of the seller's expense function u_t
  (eq. for u_t in Section 3; payoff (0, 0) at the extra time N+1, Section
  4.1; no cost at t = 0).
* ``bid_enum``: for every stopping time tau of the path tree with values in
  0..N+1, maximise the amount x the buyer can borrow, i.e. start from (-x, 0)
  and reach the epigraph of the buyer's expense function at tau; the bid is
  the largest of these.

Neither uses any recursion over the recombining tree, so agreement with the
oracle's backward induction is an independent check.  ``infconv_brute`` is the
rebalancing restriction of Section 3 evaluated by brute force.
"""
import math
from decimal import Context, Decimal

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

PUT, CALL, BULL, PUT_CASH, CALL_CASH, BEAR, STRADDLE = 0, 1, 2, 3, 4, 5, 6
EUROPEAN, COST_AT_T0 = 1, 2


def _kt(k, t, flags):
    """Cost rate at time t: none at t = 0 (Section 4.1) unless the variant
    charges it there too."""
    return k if (t >= 1 or (flags & COST_AT_T0)) else 0.0


def _exercisable(t, N, flags):
    """Times at which the holder may exercise: 0..N for the American option,
    N only for the European variant; never at the extra time N+1."""
    return t == N if (flags & EUROPEAN) else t <= N


def _payoff(pay, S, K, K2):
    """(xi, zeta) of Section 3: the holder receives xi in cash and zeta
    shares.  Put (K, -1) and call (-K, 1) by delivery; in cash: bull spread
    (S-K)^+ - (S-K2)^+, put (K-S)^+, call (S-K)^+, bear spread
    (K2-S)^+ - (K-S)^+, straddle |S-K|."""
    if pay == PUT:
        return K, -1.0
    if pay == CALL:
        return -K, 1.0
    if pay == BULL:
        return max(S - K, 0.0) - max(S - K2, 0.0), 0.0
    if pay == PUT_CASH:
        return max(K - S, 0.0), 0.0
    if pay == CALL_CASH:
        return max(S - K, 0.0), 0.0
    if pay == BEAR:
        return max(K2 - S, 0.0) - max(K - S, 0.0), 0.0
    return abs(S - K), 0.0


def exp_nearest(x):
    """e^x as the binary64 number nearest to it (Section 4.1's u and r are
    exponentials; their binary64 values are taken correctly rounded): the
    exponential in 60-digit decimal arithmetic, then Python's correctly
    rounded conversion to binary64."""
    return float(Decimal(x).exp(Context(prec=60)))


def _tree(S0, sigma, R, T, N):
    dt = T / N
    u = exp_nearest(sigma * math.sqrt(dt))
    r = exp_nearest(R * dt)
    return u, r


def _nodes(N):
    """Path-tree nodes of times 0..N+1 in breadth-first order: node i has
    children 2i+1 (up) and 2i+2 (down); returns (time, ups) per node."""
    out = [(0, 0)]
    for i in range(2 ** (N + 2) - 1):
        t, j = out[i]
        if t < N + 1:
            out.append((t + 1, j + 1))
            out.append((t + 1, j))
    return out[: 2 ** (N + 2) - 1]


def ask_lp(S0, K, R, sigma, T, k, N, payoff=PUT, K2=0.0, flags=0, with_hedge=False):
    """Seller's superhedging price by linear programming on the path tree.

    The portfolio that arrives at a node must cover delivery there when the
    holder may exercise at that time (every time 0..N, or N alone for the
    European variant) and must be solvent at the extra time N+1."""
    u, r = _tree(S0, sigma, R, T, N)
    nodes = _nodes(N)
    n = len(nodes)
    # variables: X_i, Y_i for every node; b_i, s_i for nodes of time <= N
    trade = [i for i, (t, _) in enumerate(nodes) if t <= N]
    tidx = {i: q for q, i in enumerate(trade)}
    nv = 2 * n + 2 * len(trade)
    X = lambda i: 2 * i
    Y = lambda i: 2 * i + 1
    B = lambda i: 2 * n + 2 * tidx[i]
    Sv = lambda i: 2 * n + 2 * tidx[i] + 1
    eq_r, eq_c, eq_v, beq = [], [], [], []
    row = 0

    def add(rw, col, val):
        eq_r.append(rw); eq_c.append(col); eq_v.append(val)

    add(row, Y(0), 1.0); beq.append(0.0); row += 1
    for i in trade:
        t, j = nodes[i]
        S = S0 * u ** (2 * j - t)
        kt = _kt(k, t, flags)
        Sa, Sb = (1 + kt) * S, (1 - kt) * S
        for c in (2 * i + 1, 2 * i + 2):
            # X_c = r (X_i - Sa b_i + Sb s_i)
            add(row, X(c), 1.0); add(row, X(i), -r); add(row, B(i), r * Sa); add(row, Sv(i), -r * Sb)
            beq.append(0.0); row += 1
            # Y_c = Y_i + b_i - s_i
            add(row, Y(c), 1.0); add(row, Y(i), -1.0); add(row, B(i), -1.0); add(row, Sv(i), 1.0)
            beq.append(0.0); row += 1
    Aeq = sp.csr_matrix((eq_v, (eq_r, eq_c)), shape=(row, nv))
    ub_r, ub_c, ub_v, bub = [], [], [], []
    row = 0
    for i, (t, j) in enumerate(nodes):
        if not (_exercisable(t, N, flags) or t == N + 1):
            continue
        S = S0 * u ** (2 * j - t)
        kt = _kt(k, t, flags)
        Sa, Sb = (1 + kt) * S, (1 - kt) * S
        xi, ze = _payoff(payoff, S, K, K2) if t <= N else (0.0, 0.0)
        for Sx in (Sa, Sb):
            # X_i >= xi - Sx (Y_i - ze)  <=>  -X_i - Sx Y_i <= -xi - Sx ze
            ub_r += [row, row]; ub_c += [X(i), Y(i)]; ub_v += [-1.0, -Sx]
            bub.append(-xi - Sx * ze); row += 1
    Aub = sp.csr_matrix((ub_v, (ub_r, ub_c)), shape=(row, nv))
    c = np.zeros(nv); c[X(0)] = 1.0
    bounds = [(None, None)] * (2 * n) + [(0, None)] * (2 * len(trade))
    res = linprog(c, A_ub=Aub, b_ub=bub, A_eq=Aeq, b_eq=beq, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError("ask LP failed: " + res.message)
    if with_hedge:
        # the holding the optimal portfolio carries from t = 0 to t = 1
        return res.fun, res.x[Y(1)]
    return res.fun


def crr_values(S0, K, R, sigma, T, N, payoff=PUT, K2=0.0, level=1):
    """The zero-cost American values V_t(c) at one level of the N-step tree
    and its stock prices: V_N = max(xi + zeta S, 0), V_t = max(xi + zeta S,
    (p V_t+1(c+1) + (1-p) V_t+1(c)) / r) (Section 3), for t = level."""
    u, r = _tree(S0, sigma, R, T, N)
    d = 1.0 / u
    p = (r - d) / (u - d)
    S = lambda t, c: S0 * u ** (2 * c - t)
    ex = lambda t, c: max(sum(np.multiply(_payoff(payoff, S(t, c), K, K2), (1.0, S(t, c)))), 0.0)
    V = [ex(N, c) for c in range(N + 1)]
    for t in range(N - 1, level - 1, -1):
        V = [max(ex(t, c), (p * V[c + 1] + (1 - p) * V[c]) / r) for c in range(t + 1)]
    return V, [S(level, c) for c in range(level + 1)]


def crr_exercise(S0, K, R, sigma, T, N, payoff=PUT, K2=0.0, flags=0):
    """The zero-cost stopping region of the tree with its extra level N+1 of
    payoff (0, 0) (Section 3 and Section 4.1): exercise at (t, c) is optimal
    when xi + zeta S >= the continuation value, which is 0 at t = N (the
    extra level) and rho (p V_t+1(c+1) + (1-p) V_t+1(c)) before, with
    V = max(xi + zeta S, continuation).  European: no exercise before N.
    Returns (flags, margins) as arrays in node order t(t+1)/2 + c; margin =
    exercise value minus continuation."""
    u, r = _tree(S0, sigma, R, T, N)
    d = 1.0 / u
    p = (r - d) / (u - d)
    euro = bool(flags & EUROPEAN)
    P = (N + 1) * (N + 2) // 2
    flg = np.zeros(P, dtype=np.uint8)
    mrg = np.zeros(P)
    S = lambda t, c: S0 * u ** (2 * c - t)
    ex = lambda t, c: float(sum(np.multiply(_payoff(payoff, S(t, c), K, K2), (1.0, S(t, c)))))
    V = None
    for t in range(N, -1, -1):
        Vt = []
        for c in range(t + 1):
            cont = 0.0 if t == N else (p * V[c + 1] + (1 - p) * V[c]) / r
            e = ex(t, c)
            allowed = not (euro and t < N)
            i = t * (t + 1) // 2 + c
            flg[i] = 1 if (allowed and e >= cont) else 0
            mrg[i] = e - cont
            Vt.append(max(e, cont) if allowed else cont)
        V = Vt
    return flg, mrg


def _stopping_times(N, flags=0):
    """All stopping times of the path tree with values in 0..N+1, each as the
    set of path-tree node indices at which the buyer exercises (N+1 means the
    option is left unexercised, payoff (0, 0)).  For the European variant
    the buyer can stop only at N or N+1."""
    def rec(i, t):
        if t == N + 1:
            return [(i,)]
        out = [(i,)] if _exercisable(t, N, flags) else []
        for a in rec(2 * i + 1, t + 1):
            for b in rec(2 * i + 2, t + 1):
                out.append(a + b)
        return out
    return rec(0, 0)


def _bid_for(stop, nodes, S0, u, r, K, K2, k, N, payoff, flags=0):
    """The most the buyer can borrow at t = 0 against exercising at the
    stopping time `stop`: start from (-x, 0), trade at (1 + k_t) S and
    (1 - k_t) S at every node strictly before the stopping time, and arrive
    at each stopping node in the epigraph of the buyer's expense function
    (payoff (0, 0) at N+1)."""
    stop = set(stop)
    # nodes strictly before tau: those with a stopping node strictly below them
    live = set()
    for i in stop:
        p = i
        while p > 0:
            p = (p - 1) // 2
            live.add(p)
    used = sorted(live | stop)
    idx = {i: q for q, i in enumerate(used)}
    tr = sorted(live)
    tix = {i: q for q, i in enumerate(tr)}
    nv = 2 * len(used) + 2 * len(tr)
    X = lambda i: 2 * idx[i]
    Y = lambda i: 2 * idx[i] + 1
    B = lambda i: 2 * len(used) + 2 * tix[i]
    Sv = lambda i: 2 * len(used) + 2 * tix[i] + 1
    er, ec, ev, beq = [], [], [], []
    row = 0
    er.append(row); ec.append(Y(0)); ev.append(1.0); beq.append(0.0); row += 1
    for i in tr:
        t, j = nodes[i]
        S = S0 * u ** (2 * j - t)
        kt = _kt(k, t, flags)
        Sa, Sb = (1 + kt) * S, (1 - kt) * S
        for c in (2 * i + 1, 2 * i + 2):
            er += [row] * 4; ec += [X(c), X(i), B(i), Sv(i)]; ev += [1.0, -r, r * Sa, -r * Sb]
            beq.append(0.0); row += 1
            er += [row] * 4; ec += [Y(c), Y(i), B(i), Sv(i)]; ev += [1.0, -1.0, -1.0, 1.0]
            beq.append(0.0); row += 1
    Aeq = sp.csr_matrix((ev, (er, ec)), shape=(row, nv))
    ur, uc, uv, bub = [], [], [], []
    row = 0
    for i in sorted(stop):
        t, j = nodes[i]
        S = S0 * u ** (2 * j - t)
        kt = _kt(k, t, flags)
        Sa, Sb = (1 + kt) * S, (1 - kt) * S
        xi, ze = _payoff(payoff, S, K, K2) if t <= N else (0.0, 0.0)
        for Sx in (Sa, Sb):
            # buyer: X >= -xi - Sx (Y + ze)  <=>  -X - Sx Y <= xi + Sx ze
            ur += [row, row]; uc += [X(i), Y(i)]; uv += [-1.0, -Sx]
            bub.append(xi + Sx * ze); row += 1
    Aub = sp.csr_matrix((uv, (ur, uc)), shape=(row, nv))
    # maximise borrowed x with X_root = -x  <=>  minimise X_root
    c = np.zeros(nv); c[X(0)] = 1.0
    bounds = [(None, None)] * (2 * len(used)) + [(0, None)] * (2 * len(tr))
    res = linprog(c, A_ub=Aub, b_ub=bub, A_eq=Aeq, b_eq=beq, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError("bid LP failed: " + res.message)
    return -res.fun


def _bid_chunk(args):
    stops, S0, K, R, sigma, T, k, N, payoff, K2, flags = args
    u, r = _tree(S0, sigma, R, T, N)
    nodes = _nodes(N)
    return max(_bid_for(s, nodes, S0, u, r, K, K2, k, N, payoff, flags) for s in stops)


def bid_enum(S0, K, R, sigma, T, k, N, payoff=PUT, K2=0.0, flags=0, workers=1):
    """Buyer's price: the best over all stopping times of the path tree of the
    amount that can be borrowed against exercising at that stopping time.
    ``workers`` > 1 spreads the linear programs over processes (the value is
    the same: a maximum)."""
    stops = _stopping_times(N, flags)
    if workers <= 1:
        return _bid_chunk((stops, S0, K, R, sigma, T, k, N, payoff, K2, flags))
    import multiprocessing as mp
    step = max(1, len(stops) // (8 * workers))
    jobs = [(stops[i:i + step], S0, K, R, sigma, T, k, N, payoff, K2, flags) for i in range(0, len(stops), step)]
    with mp.get_context("fork").Pool(workers) as pool:
        return max(pool.map(_bid_chunk, jobs))


def count_stopping_times(N):
    f = 1
    for _ in range(N + 1):
        f = 1 + f * f
    return f


def pwl_eval_np(F, y):
    """Evaluate a PWL function (x, v, s) at points y (numpy), using the same
    piece convention as the paper's piecewise definitions: on
    (x[i-1], x[i]) the slope is s[i]."""
    x, v, s = (np.asarray(a, dtype=np.float64) for a in F)
    y = np.asarray(y, dtype=np.float64)
    i = np.searchsorted(x, y, side="right")
    left = i == 0
    j = np.where(left, 0, i - 1)
    return np.where(left, v[0] + s[0] * (y - x[0]), v[j] + s[i] * (y - x[j]))


def infconv_brute(F, Sa, Sb, y):
    """v(y) = inf over delta of F(y + delta) + Sa delta^+ - Sb delta^-, the
    cheapest rebalancing of a holding y at ask Sa / bid Sb (Section 3).  The
    infimum of a PWL function plus a two-slope cone is attained at delta = 0
    or where y + delta is a breakpoint of F, so this is exact."""
    x = np.asarray(F[0], dtype=np.float64)
    vx = pwl_eval_np(F, x)
    y = np.asarray(y, dtype=np.float64)
    delta = x[None, :] - y[:, None]
    cost = np.where(delta >= 0, Sa * delta, Sb * delta)
    return np.minimum(pwl_eval_np(F, y), (vx[None, :] + cost).min(axis=1))
