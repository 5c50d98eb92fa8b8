"""Seeded synthetic option books shaped like the paper's workloads.

This module only draws parameters; it holds none of the pricing arithmetic,
so both the product path and the CPU oracle can take their inputs from it.

The paper prices single options (Section 5: put and bull spread with
T = 0.25, sigma = 0.2, R = 0.1 and N up to 1500; Appendix: put with T = 3,
sigma = 0.3, R = 0.06 and N up to 40000).  The books below stand in for
those workloads at the sizes used by the tests and the benchmark.
"""
import numpy as np

PUT, CALL, BULL, PUT_CASH, CALL_CASH, BEAR, STRADDLE = 0, 1, 2, 3, 4, 5, 6
EUROPEAN, COST_AT_T0 = 1, 2

# Layout of bt_params in include/bt.h (72 bytes).
PARAMS_DTYPE = np.dtype([
    ("S0", "<f8"), ("K", "<f8"), ("K2", "<f8"), ("R", "<f8"), ("sigma", "<f8"),
    ("T", "<f8"), ("k", "<f8"), ("N", "<i4"), ("payoff", "<i4"),
    ("flags", "<u4"), ("reserved", "<u4"),
])
assert PARAMS_DTYPE.itemsize == 72

# Layout of bt_result (56 bytes) and bt_grad (64 bytes).
RESULT_DTYPE = np.dtype([
    ("ask", "<f8"), ("bid", "<f8"), ("price0", "<f8"),
    ("bp_total_ask", "<i8"), ("bp_total_bid", "<i8"),
    ("bp_max_ask", "<i4"), ("bp_max_bid", "<i4"),
    ("status", "<i4"), ("reserved", "<i4"),
])
assert RESULT_DTYPE.itemsize == 56
GRAD_DTYPE = np.dtype([(f"{side}_{g}", "<f8") for side in ("ask", "bid")
                       for g in ("dS0", "dsigma", "dR", "dk")])
assert GRAD_DTYPE.itemsize == 64
# Layout of bt_hedge (32 bytes).
HEDGE_DTYPE = np.dtype([("ask_lo", "<f8"), ("ask_hi", "<f8"), ("bid_lo", "<f8"), ("bid_hi", "<f8")])


def book(rows):
    """A book from an iterable of dicts (missing K2 / flags default to 0)."""
    rows = list(rows)
    b = np.zeros(len(rows), dtype=PARAMS_DTYPE)
    for i, r in enumerate(rows):
        for key in ("S0", "K", "K2", "R", "sigma", "T", "k", "N", "payoff", "flags"):
            b[i][key] = r.get(key, 0)
    return b


def single_put_n100():
    """American put, N = 100, S0 = K = 100, R = 0.05, sigma = 0.2, T = 1,
    k = 0.005 (the small single-tree case)."""
    return book([dict(S0=100.0, K=100.0, R=0.05, sigma=0.2, T=1.0, k=0.005, N=100, payoff=PUT)])


def paper_grid(N):
    """Single American puts and calls, S0 = 100, K in {90, 100, 110},
    R = 0.05, sigma = 0.3, T = 1, k in {0, 0.0025, 0.005, 0.01}: 24 trees of
    N steps (paper-scale single trees, Section 5 sizes)."""
    rows = []
    for pay in (PUT, CALL):
        for K in (90.0, 100.0, 110.0):
            for k in (0.0, 0.0025, 0.005, 0.01):
                rows.append(dict(S0=100.0, K=K, R=0.05, sigma=0.3, T=1.0, k=k, N=N, payoff=pay))
    return book(rows)


def mixed_book(n=4096, seed=3, n_lo=200, n_hi=2000):
    """Mixed book: payoff put/call/bull spread at 40/40/20 % (bull spread
    K2 = K U[1.05, 1.3]); N uniform integer in [n_lo, n_hi];
    S0 = 100 exp(0.2 Z); K = S0 U[0.8, 1.2]; sigma U[0.1, 0.6]; T U[0.1, 2];
    R U[0, 0.08]; k U[0, 0.02].  Draws in this order, each a vector of n."""
    g = np.random.Generator(np.random.PCG64(seed))
    u = g.random(n)
    payoff = np.where(u < 0.4, PUT, np.where(u < 0.8, CALL, BULL)).astype(np.int32)
    N = g.integers(n_lo, n_hi, size=n, endpoint=True).astype(np.int32)
    S0 = 100.0 * np.exp(0.2 * g.standard_normal(n))
    K = S0 * g.uniform(0.8, 1.2, n)
    K2 = K * g.uniform(1.05, 1.3, n)
    sigma = g.uniform(0.1, 0.6, n)
    T = g.uniform(0.1, 2.0, n)
    R = g.uniform(0.0, 0.08, n)
    k = g.uniform(0.0, 0.02, n)
    b = np.zeros(n, dtype=PARAMS_DTYPE)
    b["S0"], b["K"], b["K2"], b["R"], b["sigma"], b["T"], b["k"] = S0, K, K2, R, sigma, T, k
    b["N"], b["payoff"] = N, payoff
    b["K2"] = np.where(payoff == BULL, K2, 0.0)
    return b


def greeks_book(n=1024, seed=4):
    """The mixed book's generator with N uniform in [500, 1500]."""
    return mixed_book(n=n, seed=seed, n_lo=500, n_hi=1500)


def stress_book(n=16384, seed=5):
    """Stress book: N = round(exp(U[ln 64, ln 8192])), k U[0, 0.02], S0 = 100,
    R = 0.05, sigma = 0.3, T = 1, K uniform on {90, 100, 110}, payoffs
    40/40/20 with bull K2 = K U[1.05, 1.3]."""
    g = np.random.Generator(np.random.PCG64(seed))
    u = g.random(n)
    payoff = np.where(u < 0.4, PUT, np.where(u < 0.8, CALL, BULL)).astype(np.int32)
    N = np.rint(np.exp(g.uniform(np.log(64), np.log(8192), n))).astype(np.int32)
    k = g.uniform(0.0, 0.02, n)
    K = g.choice(np.array([90.0, 100.0, 110.0]), n)
    K2 = K * g.uniform(1.05, 1.3, n)
    b = np.zeros(n, dtype=PARAMS_DTYPE)
    b["S0"], b["K"], b["R"], b["sigma"], b["T"], b["k"] = 100.0, K, 0.05, 0.3, 1.0, k
    b["N"], b["payoff"] = N, payoff
    b["K2"] = np.where(payoff == BULL, K2, 0.0)
    return b


def long_put():
    """One American put with N = 20000, S0 = K = 100, sigma = 0.4, T = 2,
    R = 0.05, k = 0.01 (long tree)."""
    return book([dict(S0=100.0, K=100.0, R=0.05, sigma=0.4, T=2.0, k=0.01, N=20000, payoff=PUT)])


def random_small(n, seed, n_max=300):
    """Small random options for parity tests: every payoff and flag, costs
    from zero to 10 %, N from 1 to n_max."""
    g = np.random.Generator(np.random.PCG64(seed))
    b = np.zeros(n, dtype=PARAMS_DTYPE)
    for i in range(n):
        pay = int(g.integers(0, 3))
        S0 = 100 * np.exp(0.2 * g.standard_normal())
        K = S0 * g.uniform(0.8, 1.2)
        k = float(g.choice([0.0, g.uniform(0, 0.02), g.uniform(0, 0.1)]))
        b[i] = (S0, K, K * g.uniform(1.05, 1.3) if pay == BULL else 0.0, g.uniform(0, 0.08),
                g.uniform(0.1, 0.6), g.uniform(0.1, 2.0), k, int(g.integers(1, n_max + 1)), pay,
                int(g.choice([0, 0, 0, EUROPEAN, COST_AT_T0])), 0)
    return b


def variants_book(n, seed, n_max=200):
    """Every payoff shape (delivered and cash-settled puts and calls, bull
    and bear spreads, straddles), every flag, costs from zero to 10 %, N from
    1 to n_max; payoff = index mod 7 so that each shape appears."""
    g = np.random.Generator(np.random.PCG64(seed))
    b = np.zeros(n, dtype=PARAMS_DTYPE)
    for i in range(n):
        pay = i % 7
        S0 = 100 * np.exp(0.2 * g.standard_normal())
        K = S0 * g.uniform(0.8, 1.2)
        k = float(g.choice([0.0, g.uniform(0, 0.02), g.uniform(0, 0.1)]))
        b[i] = (S0, K, K * g.uniform(1.05, 1.3) if pay in (BULL, BEAR) else 0.0, g.uniform(0, 0.08),
                g.uniform(0.1, 0.6), g.uniform(0.1, 2.0), k, int(g.integers(1, n_max + 1)), pay,
                int(g.choice([0, 0, 0, EUROPEAN, COST_AT_T0])), 0)
    return b


def nodes(b):
    """Tree nodes sum (N+1)(N+2)/2 of a book (levels 0..N)."""
    N = b["N"].astype(np.int64)
    return int(((N + 1) * (N + 2) // 2).sum())


def greeks_fd_subset(n=1024):
    """The 32 options of the Greeks book that the finite-difference and the
    tangent checks use: PCG64(44).choice(n, 32) without replacement."""
    return np.sort(np.random.Generator(np.random.PCG64(44)).choice(n, 32, replace=False))


def stress_sample(s):
    """Indices of a seeded sample of a stress book spanning its N range:
    8 costly calls and bull spreads (N >= 4000, k >= 1 %), and 8 options from
    each of the N bands [64, 256), [256, 2048), [2048, 8192] (any payoff),
    drawn with PCG64(56) in that order."""
    g = np.random.Generator(np.random.PCG64(56))
    N, k, pay = s["N"], s["k"], s["payoff"]
    heavy = np.flatnonzero((N >= 4000) & (k >= 0.01) & (pay != PUT))
    pick = [g.choice(heavy, 8, replace=False)]
    for lo, hi in ((64, 256), (256, 2048), (2048, 8193)):
        band = np.setdiff1d(np.flatnonzero((N >= lo) & (N < hi)), pick[0])
        pick.append(g.choice(band, 8, replace=False))
    return np.sort(np.concatenate(pick))
