"""Brute-force pins of the oracle's piecewise-linear operations (no GPU).

MERGE is checked against the pointwise max/min of independently evaluated
inputs; CLIP and ENV against the rebalancing restriction of Section 3
evaluated by brute force (``definitions.infconv_brute``)."""
import numpy as np
import pytest

import oracle
from oracle import definitions as D


def rand_pwl(rng, m, convex=False, lo=-5.0, hi=5.0, smin=-150.0, smax=-20.0):
    x = np.sort(rng.uniform(lo, hi, m))
    while np.any(np.diff(x) <= 0):
        x = np.sort(rng.uniform(lo, hi, m))
    s = rng.uniform(smin, smax, m + 1)
    if convex:
        s = np.sort(s)
    v = np.empty(m)
    v[0] = rng.uniform(-50, 50)
    for j in range(1, m):
        v[j] = v[j - 1] + s[j] * (x[j] - x[j - 1])
    return x, v, s


def check_canonical(H):
    x, v, s = H
    assert len(s) == len(x) + 1 and len(x) >= 1
    assert np.all(np.diff(x) > 0)
    if len(x) > 1:
        assert np.all(s[:-1] != s[1:])


def grid(*fs, n=400):
    pts = np.concatenate([np.asarray(f[0]) for f in fs])
    lo, hi = pts.min() - 3.0, pts.max() + 3.0
    ys = np.concatenate([np.linspace(lo, hi, n), pts, pts + 1e-7, pts - 1e-7])
    return ys


@pytest.mark.parametrize("seed", range(40))
def test_merge_is_pointwise_max_and_min(seed):
    rng = np.random.default_rng(seed)
    F = rand_pwl(rng, int(rng.integers(1, 9)))
    G = rand_pwl(rng, int(rng.integers(1, 9)))
    for op, fn in ((oracle.MERGE_MAX, np.maximum), (oracle.MERGE_MIN, np.minimum)):
        H = oracle.pwl_op(op, F, G)
        check_canonical(H)
        ys = grid(F, G, H)
        want = fn(D.pwl_eval_np(F, ys), D.pwl_eval_np(G, ys))
        got = D.pwl_eval_np(H, ys)
        assert np.allclose(got, want, rtol=1e-11, atol=1e-9)
        # slopes are carried: every output slope is one of the input slopes
        assert set(H[2]).issubset(set(F[2]) | set(G[2]))


def test_merge_tangent_and_equal_functions():
    F = ([0.0], [0.0], [-3.0, -1.0])
    H = oracle.pwl_op(oracle.MERGE_MAX, F, F)
    assert list(H[0]) == [0.0] and list(H[2]) == [-3.0, -1.0]
    # parallel lines never cross; the larger is kept and the result is a line
    L1 = ([0.0], [1.0], [-2.0, -2.0])
    L2 = ([1.0], [0.0], [-2.0, -2.0])
    H = oracle.pwl_op(oracle.MERGE_MAX, L1, L2)
    assert len(H[0]) == 1 and H[2][0] == H[2][1] == -2.0
    assert oracle.pwl_eval(H, 0.0) == 2.0   # L2(0) = 0 + (-2)(0 - 1)


@pytest.mark.parametrize("seed", range(30))
def test_clip_is_restriction_for_convex(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(1, 10))
    F = rand_pwl(rng, m, convex=True)
    a, b = np.sort(rng.uniform(F[2][0], F[2][-1], 2))
    if a == b:
        b = a + 1.0
    # precondition of the restriction step: outer slopes outside [a, b]
    assert F[2][0] < a and F[2][-1] > b
    H = oracle.pwl_op(oracle.CLIP, F, a=a, b=b)
    check_canonical(H)
    assert H[2][0] == a and H[2][-1] == b
    assert np.all((H[2] >= a) & (H[2] <= b))
    ys = grid(F, H)
    want = D.infconv_brute(F, -a, -b, ys)
    assert np.allclose(D.pwl_eval_np(H, ys), want, rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("seed", range(60))
def test_env_is_restriction_for_nonconvex(seed):
    rng = np.random.default_rng(200 + seed)
    m = int(rng.integers(1, 14))
    F = rand_pwl(rng, m)
    s = F[2]
    a, b = np.sort(rng.uniform(-120, -40, 2))
    s[0] = min(s[0], a - rng.uniform(1, 30))
    s[-1] = max(s[-1], b + rng.uniform(1, 30))
    x = F[0]
    v = np.empty(m)
    v[0] = F[1][0]
    for j in range(1, m):
        v[j] = v[j - 1] + s[j] * (x[j] - x[j - 1])
    F = (x, v, s)
    H = oracle.pwl_op(oracle.ENV, F, a=a, b=b)
    check_canonical(H)
    assert H[2][0] == a and H[2][-1] == b
    assert np.all((H[2] >= a) & (H[2] <= b))
    ys = grid(F, H)
    want = D.infconv_brute(F, -a, -b, ys)
    got = D.pwl_eval_np(H, ys)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-8), np.max(np.abs(got - want))


@pytest.mark.parametrize("seed", range(120))
def test_env_degenerate_slopes_and_ties(seed):
    # pieces with slope exactly a or b make h = v - a x tie between
    # neighbouring points and put crossings on piece ends; the result must
    # still be the restriction (values; 1-ulp slivers are allowed)
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(2, 30))
    x = np.sort(rng.uniform(-5, 5, m))
    if np.any(np.diff(x) <= 0):
        return
    a, b = np.sort(rng.uniform(-120, -40, 2))
    s = rng.uniform(-150, -20, m + 1)
    u = rng.random(m + 1)
    s[u < 0.15] = a
    s[(u >= 0.15) & (u < 0.3)] = b
    s[0] = min(s[0], a - rng.uniform(1, 30))
    s[-1] = max(s[-1], b + rng.uniform(1, 30))
    v = np.empty(m)
    v[0] = rng.uniform(-50, 50)
    for j in range(1, m):
        v[j] = v[j - 1] + s[j] * (x[j] - x[j - 1])
    F = (x, v, s)
    H = oracle.pwl_op(oracle.ENV, F, a=a, b=b)
    assert np.all(np.diff(H[0]) > 0)
    assert H[2][0] == a and H[2][-1] == b
    ys = np.concatenate([np.linspace(x.min() - 3, x.max() + 3, 300), x, H[0]])
    want = D.infconv_brute(F, -a, -b, ys)
    got = D.pwl_eval_np(H, ys)
    assert np.all(np.abs(got - want) <= 1e-10 * (1 + np.abs(want)))
    # the two halves: A has slopes >= a (buying), B slopes <= b (selling)
    A = oracle.pwl_op(oracle.ENV_A, F, a=a, b=b)
    B = oracle.pwl_op(oracle.ENV_B, F, a=a, b=b)
    assert A[2][0] == a and B[2][-1] == b
    ya = np.concatenate([ys, A[0]])
    hA = np.array([min(D.pwl_eval_np(F, np.array([yy]))[0] - a * yy,
                       (D.pwl_eval_np(F, x[x >= yy]) - a * x[x >= yy]).min() if np.any(x >= yy) else np.inf)
                   for yy in ya]) + a * ya
    assert np.allclose(D.pwl_eval_np(A, ya), hA, rtol=1e-10, atol=1e-8)


@pytest.mark.parametrize("seed", range(20))
def test_env_equals_clip_on_convex(seed):
    rng = np.random.default_rng(300 + seed)
    F = rand_pwl(rng, int(rng.integers(1, 8)), convex=True)
    a, b = np.sort(rng.uniform(F[2][0], F[2][-1], 2))
    if a == b:
        b = a + 1.0
    H1 = oracle.pwl_op(oracle.CLIP, F, a=a, b=b)
    H2 = oracle.pwl_op(oracle.ENV, F, a=a, b=b)
    ys = grid(F, H1, H2)
    assert np.allclose(D.pwl_eval_np(H1, ys), D.pwl_eval_np(H2, ys), rtol=1e-11, atol=1e-9)


def test_restriction_with_equal_bounds_is_a_line():
    # no cost at t = 0 (Section 4.1): S^a_0 = S^b_0, so v_0 is a line of slope -S0
    x = np.array([-1.0, 0.5, 2.0])
    s = np.array([-60.0, -14.0, -4.0 / 3.0, 5.0])
    v = np.array([10.0, 10.0 - 14.0 * 1.5, 10.0 - 14.0 * 1.5 - 2.0])
    F = (x, v, s)
    a = -10.0
    for op in (oracle.CLIP, oracle.ENV):
        H = oracle.pwl_op(op, F, a=a, b=a)
        assert len(H[0]) == 1 and H[2][0] == H[2][1] == a
        ys = np.linspace(-4, 4, 50)
        want = D.infconv_brute(F, -a, -a, ys)
        assert np.allclose(D.pwl_eval_np(H, ys), want, rtol=1e-12, atol=1e-10)


def test_canon_drops_points_without_kink():
    F = ([0.0, 1.0, 2.0], [0.0, -1.0, -2.0], [-1.0, -1.0, -1.0, -3.0])
    H = oracle.pwl_op(oracle.CANON, F)
    assert list(H[0]) == [2.0] and list(H[2]) == [-1.0, -3.0]
    L = ([0.0, 1.0], [5.0, 4.0], [-1.0, -1.0, -1.0])
    H = oracle.pwl_op(oracle.CANON, L)
    assert list(H[0]) == [0.0] and list(H[1]) == [5.0] and list(H[2]) == [-1.0, -1.0]


def test_eval_convention():
    F = ([0.0, 1.0], [2.0, 1.0], [-3.0, -1.0, -2.0])
    assert oracle.pwl_eval(F, -1.0) == 5.0
    assert oracle.pwl_eval(F, 0.0) == 2.0
    assert oracle.pwl_eval(F, 0.5) == 1.5
    assert oracle.pwl_eval(F, 1.0) == 1.0
    assert oracle.pwl_eval(F, 3.0) == -3.0
