"""Exact-rational recursion of Section 3 (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The seller's and buyer's recursions are run in exact rational arithmetic
(``fractions.Fraction``) from the same binary64 inputs the C oracle uses: the
stock table S0 u^j, rho = 1/r and k, converted exactly.  Nothing rounds, so
the result is the exact price of that tree and the exact expense functions,
whose genuine kinks (slope changes) are what the breakpoint counts of the
binary64 recursion approximate.

It is written from the definitions only, with none of the C oracle's
operation orders or tie rules:

* the maximum or minimum of several piecewise-linear functions is evaluated
  on every breakpoint of every operand and every crossing of two of their
  pieces; between two consecutive such abscissae no operand crosses another,
  so one operand is active on the whole interval (Section 3's w_t and z_t);
* the slope restriction of Section 3 (the cheapest rebalancing of a holding
  y at the ask (1+k)S and the bid (1-k)S) is the inf-convolution
  v(y) = inf over y' of f(y') + (1+k)S (y'-y)^+ - (1-k)S (y'-y)^-,
  whose infimum is attained at y' = y or at a breakpoint of f, so
  v = min(f, V_j over the breakpoints x_j), V_j the cone with vertex
  (x_j, f(x_j)) and slopes a = -(1+k)S to the left, b = -(1-k)S to the right.
  This is the definition for both parties; the seller's convex case needs no
  special treatment.

Sizes: the rationals grow with the depth of the tree, so this is for small
trees (N up to about 30).
"""
from fractions import Fraction

PUT, CALL, BULL, PUT_CASH, CALL_CASH, BEAR, STRADDLE = 0, 1, 2, 3, 4, 5, 6
EUROPEAN, COST_AT_T0 = 1, 2


class Pwl:
    """Continuous piecewise-linear function: strictly increasing points xs
    with values vs; slopes ss[0] left of xs[0], ss[j] on (xs[j-1], xs[j]),
    ss[m] right of xs[-1].  Canonical: no point with equal slopes on both
    sides, except the single anchor point of a line."""

    __slots__ = ("xs", "vs", "ss")

    def __init__(self, xs, vs, ss):
        self.xs, self.vs, self.ss = list(xs), list(vs), list(ss)

    def __call__(self, y):
        xs = self.xs
        # i = number of points <= y
        lo, hi = 0, len(xs)
        while lo < hi:
            mid = (lo + hi) // 2
            if xs[mid] <= y:
                lo = mid + 1
            else:
                hi = mid
        if lo == 0:
            return self.vs[0] + self.ss[0] * (y - xs[0])
        return self.vs[lo - 1] + self.ss[lo] * (y - xs[lo - 1])

    def pieces(self):
        """(lo, hi, slope, intercept) of every piece; lo/hi None = unbounded."""
        xs, vs, ss = self.xs, self.vs, self.ss
        out = []
        for i in range(len(xs) + 1):
            lo = xs[i - 1] if i > 0 else None
            hi = xs[i] if i < len(xs) else None
            ref = i - 1 if i > 0 else 0
            out.append((lo, hi, ss[i], vs[ref] - ss[i] * xs[ref]))
        return out

    def kinks(self):
        """Genuine breakpoints: the number of slope changes."""
        return sum(1 for j in range(len(self.xs)) if self.ss[j] != self.ss[j + 1])


def vee(x0, v0, sl, sr):
    return Pwl([x0], [v0], [sl, sr])


def canonical(xs, vs, ss):
    """Drops every point whose two slopes are equal; a line keeps one point."""
    kx, kv, ks = [], [], [ss[0]]
    for j in range(len(xs)):
        if ss[j] != ss[j + 1]:
            kx.append(xs[j]); kv.append(vs[j]); ks.append(ss[j + 1])
    if not kx:
        return Pwl([xs[0]], [vs[0]], [ss[0], ss[0]])
    return Pwl(kx, kv, ks)


def _overlap(p, q):
    lo = p[0] if q[0] is None else (q[0] if p[0] is None else max(p[0], q[0]))
    hi = p[1] if q[1] is None else (q[1] if p[1] is None else min(p[1], q[1]))
    return lo, hi


def envelope(fs, op):
    """Pointwise max (op = max) or min (op = min) of the functions fs."""
    cand = set()
    for f in fs:
        cand.update(f.xs)
    pieces = [f.pieces() for f in fs]
    for a in range(len(fs)):
        for b in range(a + 1, len(fs)):
            for p in pieces[a]:
                for q in pieces[b]:
                    if p[2] == q[2]:
                        continue
                    y = (q[3] - p[3]) / (p[2] - q[2])
                    lo, hi = _overlap(p, q)
                    if (lo is None or y >= lo) and (hi is None or y <= hi):
                        cand.add(y)
    P = sorted(cand)

    def best_at(y):
        vals = [f(y) for f in fs]
        w = op(vals)
        return w, [i for i, v in enumerate(vals) if v == w]

    def slope_on(y, side_slopes):
        # the active operand on an interval without crossings: the best value
        # at an interior point; equal best values there mean the same line
        _, idx = best_at(y)
        return side_slopes(idx[0])

    vs = [op(f(y) for f in fs) for y in P]
    # left of P[0] every operand is on its left tail
    ss = [slope_on(P[0] - 1, lambda i: fs[i].ss[0])]
    for j in range(len(P) - 1):
        mid = (P[j] + P[j + 1]) / 2

        def sl(i, mid=mid):
            f = fs[i]
            # slope of f at an interior point of its piece holding mid
            k = sum(1 for x in f.xs if x <= mid)
            return f.ss[k]
        ss.append(slope_on(mid, sl))
    ss.append(slope_on(P[-1] + 1, lambda i: fs[i].ss[-1]))
    return canonical(P, vs, ss)


def restrict(f, a, b):
    """Largest minorant of f with slopes in [a, b] (a <= b): the cheapest
    rebalancing at the ask -a and the bid -b (Section 3)."""
    cones = [vee(x, v, a, b) for x, v in zip(f.xs, f.vs)]
    return envelope([f] + cones, min)


def _payoff(pay, S, K, K2):
    """(xi, zeta) of Section 3 for every payoff shape; works on Fractions and
    on floats alike."""
    zero = S - S
    if pay == PUT:
        return K, zero - 1
    if pay == CALL:
        return -K, zero + 1
    if pay == BULL:
        return max(S - K, zero) - max(S - K2, zero), zero
    if pay == PUT_CASH:
        return max(K - S, zero), zero
    if pay == CALL_CASH:
        return max(S - K, zero), zero
    if pay == BEAR:
        return max(K2 - S, zero) - max(K - S, zero), zero
    return abs(S - K), zero


def _node_constants(S, kt, pay, K, K2, rounded):
    """a = -(1+k_t) S, b = -(1-k_t) S and the payoff (xi, zeta) at a node:
    exact, or (rounded) the binary64 values of the same formulas."""
    if not rounded:
        one = Fraction(1)
        xi, ze = _payoff(pay, S, K, K2)
        return -(one + kt) * S, -(one - kt) * S, xi, ze
    s, k_, K_, K2_ = float(S), float(kt), float(K), float(K2)
    a, b = -((1.0 + k_) * s), -((1.0 - k_) * s)
    xi, ze = _payoff(pay, s, K_, K2_)
    return Fraction(a), Fraction(b), Fraction(xi), Fraction(ze)


def side_price(stock, rho, k, N, pay, K, K2, side, flags=0, rounded=True, exmap=None):
    """Exact recursion of one party (0 seller, 1 buyer) over levels N+1..0.
    stock(j) = S0 u^j as a Fraction.  rounded: the node constants a, b, xi,
    zeta (and the slopes of level N+1) are the binary64 values of their
    formulas, as in the C oracle, so that only the recursion's own
    operations (maximum, discount, restriction, exercise) are exact.
    Returns (root value z_0(0) as a Fraction, total genuine kinks over levels
    0..N, largest count).  exmap (a dict, optional) receives for every node
    (t, c) at which exercise is allowed the pair (u_t(0), v_t(0)): the
    party's expense at zero stock holding if it exercises there, and if it
    goes on."""
    cur = []
    for c in range(N + 2):
        a, b, _, _ = _node_constants(stock(2 * c - (N + 1)), k, pay, K, K2, rounded)
        cur.append(vee(Fraction(0), Fraction(0), a, b))
    tot = mx = 0
    for t in range(N, -1, -1):
        kt = k if (t >= 1 or (flags & COST_AT_T0)) else Fraction(0)
        nxt = []
        for c in range(t + 1):
            S = stock(2 * c - t)
            a, b, xi, ze = _node_constants(S, kt, pay, K, K2, rounded)
            w = envelope([cur[c + 1], cur[c]], max)
            f = Pwl(w.xs, [v * rho for v in w.vs], [s * rho for s in w.ss])
            v = restrict(f, a, b)
            if (flags & EUROPEAN) and t < N:
                z = v
            else:
                u = vee(ze, xi, a, b) if side == 0 else vee(-ze, -xi, a, b)
                z = envelope([u, v], max if side == 0 else min)
                if exmap is not None:
                    exmap[(t, c)] = (u(Fraction(0)), v(Fraction(0)))
            n = z.kinks()
            tot += n
            mx = max(mx, n)
            nxt.append(z)
        cur = nxt
    return cur[0](Fraction(0)), tot, mx


def price(stock_table, rho, k, N, payoff, K, K2=0.0, flags=0, rounded=True):
    """Exact ask and bid from binary64 inputs: stock_table[j + N + 1] = S0 u^j
    (j = -(N+1)..N+1), rho, k, K, K2 (all converted exactly; see side_price
    for `rounded`).  Returns a dict with Fractions ask, bid and the genuine
    kink counts per side."""
    tab = [Fraction(float(s)) for s in stock_table]

    def stock(j):
        return tab[j + N + 1]

    rho, k, K, K2 = Fraction(float(rho)), Fraction(float(k)), Fraction(float(K)), Fraction(float(K2))
    za, ta, ma = side_price(stock, rho, k, N, payoff, K, K2, 0, flags, rounded)
    zb, tb, mb = side_price(stock, rho, k, N, payoff, K, K2, 1, flags, rounded)
    return dict(ask=za, bid=-zb, kinks_total_ask=ta, kinks_total_bid=tb, kinks_max_ask=ma, kinks_max_bid=mb)
