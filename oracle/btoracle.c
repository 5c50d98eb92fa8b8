/*
 * btoracle.c -- plain CPU oracle for the ask and bid prices of an American
 * option under proportional transaction costs on a recombining CRR tree
 * (Zhang, Roux & Zastawniak 2011, "Parallel Binomial American Option Pricing
 * with (and without) Transaction Costs", Sections 3 and 4.1), plus the
 * zero-cost scalar CRR price (same paper, Section 3 and Appendix).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The product path (HIP kernels and
 * the C-ABI library) shares no code with it.
 *
 * The file is compiled twice: with NT=0 (values only, symbols *_v) and with
 * NT=4 (forward-mode tangents with respect to S0, sigma, R, k; symbols *_g).
 * Comparisons always look at values only, so both builds take the same
 * branches and produce bit-identical values.
 *
 * Everything is plain IEEE binary64 with no contraction (build with
 * -ffp-contract=off).  Every piecewise-linear (PWL) operation follows the
 * canonical definitions written out next to it; readings of the paper where
 * it is silent are listed in the design notes of the repository.
 *
 * What pins each function (a plausible mistake in it fails these tests):
 *   pwl_canon, pwl_eval      tests/test_oracle_pwl.py (points, tails, lines)
 *                            and every price test below
 *   pwl_merge                test_oracle_pwl.py (pointwise max/min on a
 *                            grid, crossings, ties); the worked example of
 *                            Section 3; the superhedging LP (N <= 8)
 *   pwl_scale                the worked example (110.1695 = 130 / 1.18)
 *   pwl_clip                 brute-force inf-convolution (test_oracle_pwl);
 *                            the LP for the ask; exact-rational recursion
 *   env_scan_a, pwl_env      brute-force inf-convolution on random
 *                            non-convex functions; stopping-time
 *                            enumeration for the bid (N <= 4); exact-rational
 *                            recursion (tests/test_oracle_exact.py, equal
 *                            breakpoint counts for puts and calls)
 *   exp_nearest              decimal arithmetic at 60 digits
 *                            (test_oracle_pins.py, model constants)
 *   model_init, upow         13.906 (Appendix); Black-Scholes convergence
 *                            and put-call parity (European, k = 0)
 *   crr_price                k = 0 ask = bid = CRR; 13.906
 *   root_hedge               the superhedging LP's root holding; the CRR
 *                            delta at k = 0 (test_oracle_hedge.py)
 *   exercise map             the exact-rational recursion's u_t(0) against
 *                            v_t(0) away from ties; the zero-cost stopping
 *                            region at k = 0; no exercise before N for the
 *                            European variant (test_oracle_exercise.py)
 *   side_price               every test above; cost at t = 0 and the
 *                            European variant against their LPs and
 *                            enumerations; level N+1 against the one-step
 *                            LP; spread monotone in k; trivial hedges
 *   tangents (NT = 4 build)  tests/test_oracle_grad.py (central differences)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef NT
#define NT 0
#endif
#define ND (NT > 0 ? NT : 1)

#if NT == 0
#define API(name) name##_v
#else
#define API(name) name##_g
#endif

/* ------------------------------------------------------------------------ */
/* Numbers: a value and NT tangents.                                         */
/* ------------------------------------------------------------------------ */
typedef struct { double v; double d[ND]; } num;

/* Count of binary64 additions, subtractions, multiplications and divisions
 * on values (tangents excluded), per thread: the algorithmic work. */
static _Thread_local uint64_t g_flops;

static num nc(double v) { num r; r.v = v; for (int i = 0; i < ND; i++) r.d[i] = 0.0; return r; }
static num nadd(num a, num b) { g_flops++; num r = nc(a.v + b.v); for (int i = 0; i < NT; i++) r.d[i] = a.d[i] + b.d[i]; return r; }
static num nsub(num a, num b) { g_flops++; num r = nc(a.v - b.v); for (int i = 0; i < NT; i++) r.d[i] = a.d[i] - b.d[i]; return r; }
static num nneg(num a) { num r = nc(-a.v); for (int i = 0; i < NT; i++) r.d[i] = -a.d[i]; return r; }
static num nmul(num a, num b)
{
    g_flops++;
    num r = nc(a.v * b.v);
    for (int i = 0; i < NT; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
static num ndiv(num a, num b)
{
    g_flops++;
    num r = nc(a.v / b.v);
    for (int i = 0; i < NT; i++) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}
/* max(a, 0): the positive part used by the bull-spread payoff. */
static num npos(num a) { return a.v > 0.0 ? a : nc(0.0); }

/* ------------------------------------------------------------------------ */
/* PWL functions.                                                            */
/*                                                                           */
/* F = (m >= 1; x[0..m-1] strictly increasing; v[j] = F(x[j]); s[0..m]).     */
/* s[0] is the slope left of x[0], s[m] the slope right of x[m-1], s[j] the  */
/* slope on (x[j-1], x[j]).  Slopes are carried, never recomputed from the   */
/* points.  A line is stored as one anchor point with s[0] == s[1].          */
/* ------------------------------------------------------------------------ */
typedef struct { int m, cap; num *x, *v, *s; } pwl;

static void pwl_reserve(pwl *f, int m)
{
    if (m + 1 <= f->cap) return;
    int cap = f->cap ? f->cap : 4;
    while (cap < m + 1) cap *= 2;
    f->x = (num *)realloc(f->x, sizeof(num) * cap);
    f->v = (num *)realloc(f->v, sizeof(num) * cap);
    f->s = (num *)realloc(f->s, sizeof(num) * cap);
    f->cap = cap;
}
static void pwl_free(pwl *f) { free(f->x); free(f->v); free(f->s); memset(f, 0, sizeof(*f)); }
static void pwl_copy(pwl *dst, const pwl *src)
{
    pwl_reserve(dst, src->m);
    dst->m = src->m;
    memcpy(dst->x, src->x, sizeof(num) * src->m);
    memcpy(dst->v, src->v, sizeof(num) * src->m);
    memcpy(dst->s, src->s, sizeof(num) * (src->m + 1));
}
static void pwl_swap(pwl *a, pwl *b) { pwl t = *a; *a = *b; *b = t; }

/* A "V": one kink at x0 with value v0, slope sa to the left, sb to the right. */
static void pwl_vee(pwl *f, num x0, num v0, num sa, num sb)
{
    pwl_reserve(f, 1);
    f->m = 1; f->x[0] = x0; f->v[0] = v0; f->s[0] = sa; f->s[1] = sb;
}

/* Number of breakpoints = number of slope changes; a line has none. */
static int pwl_bp(const pwl *f)
{
    int n = 0;
    for (int j = 0; j < f->m; j++) n += (f->s[j].v != f->s[j + 1].v);
    return n;
}

/* CANON: drop every point whose two adjacent slopes are bit-equal.  Removing
 * such a point leaves every other point's adjacent slopes unchanged, so the
 * test is local.  If nothing is left the function is a line and keeps its
 * first point as the anchor. */
static void pwl_canon(pwl *f)
{
    int m = f->m, k = 0;
    num s0 = f->s[0];
    for (int j = 0; j < m; j++) {
        if (f->s[j].v != f->s[j + 1].v) {
            f->x[k] = f->x[j]; f->v[k] = f->v[j]; f->s[k + 1] = f->s[j + 1];
            k++;
        }
    }
    f->s[0] = s0;
    if (k == 0) { /* a line: anchor at the first point (x[0], v[0] untouched) */
        f->s[1] = s0;
        k = 1;
    }
    f->m = k;
}

/* EVAL(F, y): with i = #{j : x[j] <= y}, F(y) = v[0] + s[0](y - x[0]) if
 * i = 0, else v[i-1] + s[i](y - x[i-1]).  A breakpoint returns its stored
 * value. */
static num eval_at(const pwl *f, int i, num y)
{
    if (i == 0) return nadd(f->v[0], nmul(f->s[0], nsub(y, f->x[0])));
    return nadd(f->v[i - 1], nmul(f->s[i], nsub(y, f->x[i - 1])));
}

static num pwl_eval(const pwl *f, num y)
{
    /* i = #{j : x[j] <= y} by bisection */
    int lo = 0, hi = f->m;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (f->x[mid].v <= y.v) lo = mid + 1; else hi = mid;
    }
    return eval_at(f, lo, y);
}

enum { OP_MAX = 0, OP_MIN = 1 };
enum { PICK_NONE = -1, PICK_F = 0, PICK_G = 1 };

/* Which function is better (larger for MAX, smaller for MIN) given
 * d = F - G at a point; PICK_NONE on a tie. */
static int better(int op, double d)
{
    if (op == OP_MAX) return d > 0.0 ? PICK_F : (d < 0.0 ? PICK_G : PICK_NONE);
    return d < 0.0 ? PICK_F : (d > 0.0 ? PICK_G : PICK_NONE);
}

static num opval(int op, num a, num b)
{
    if (op == OP_MAX) return a.v >= b.v ? a : b;
    return a.v <= b.v ? a : b;
}

static void push_pt(pwl *h, num x, num v, num sright)
{
    pwl_reserve(h, h->m + 1);
    h->x[h->m] = x; h->v[h->m] = v; h->s[h->m + 1] = sright;
    h->m++;
}

/*
 * MERGE(F, G, op): the pointwise maximum (max over the two children for both
 * parties, and max(u_t, v_t) for the seller) or minimum (min(u_t, v_t) for
 * the buyer) of two PWL functions, Section 3.
 *
 * 1. P = sorted union of the breakpoints of F and G, exact duplicates merged.
 *    At each P_k: d_k = EVAL(F, P_k) - EVAL(G, P_k).
 * 2. On an interval (P_k, P_k+1) with slopes sF, sG: a crossing exists iff
 *    sF != sG and d_k, d_k+1 have strictly opposite signs; then
 *    y* = P_k + d_k / (sG - sF).  If y* <= P_k the interval takes the winner
 *    at its right end, if y* >= P_k+1 the winner at its left end, otherwise
 *    y* is a new point.  Without a crossing the winner is taken at the left
 *    end, else at the right end, else by slope (MAX: the larger slope, MIN:
 *    the smaller, equal: F).
 * 3. Tails: the far winner is decided by the slopes (MAX: smaller slope on
 *    the left, larger on the right; MIN the reverse; equal slopes: by the
 *    sign of d at the end point, tie: F).  If the near-end winner differs,
 *    the crossing y* = P_ref + d_ref / (sG - sF) is added when it lies
 *    strictly outside P_ref; otherwise the whole tail takes the far winner.
 * 4. Values at output points: op(EVAL(F, y), EVAL(G, y)); slopes: those of
 *    the winner on each piece.  Then CANON.
 */
static void pwl_merge(const pwl *F, const pwl *G, int op, pwl *H)
{
    int mF = F->m, mG = G->m;
    int cap = mF + mG;
    num *P = (num *)malloc(sizeof(num) * cap);
    int *iF = (int *)malloc(sizeof(int) * cap);
    int *iG = (int *)malloc(sizeof(int) * cap);
    num *fF = (num *)malloc(sizeof(num) * cap);
    num *fG = (num *)malloc(sizeof(num) * cap);
    double *d = (double *)malloc(sizeof(double) * cap);
    int K = 0, a = 0, b = 0;
    while (a < mF || b < mG) {
        if (b >= mG || (a < mF && F->x[a].v < G->x[b].v)) { P[K] = F->x[a]; a++; }
        else if (a >= mF || G->x[b].v < F->x[a].v) { P[K] = G->x[b]; b++; }
        else { P[K] = F->x[a]; a++; b++; }
        iF[K] = a; iG[K] = b;   /* #{x <= P_k} in F and in G */
        K++;
    }
    for (int k = 0; k < K; k++) {
        fF[k] = eval_at(F, iF[k], P[k]);
        fG[k] = eval_at(G, iG[k], P[k]);
        d[k] = fF[k].v - fG[k].v;
    }

    H->m = 0;
    pwl_reserve(H, 2 * K + 1);

    /* left tail */
    {
        num sF = F->s[0], sG = G->s[0];
        int b0 = better(op, d[0]);
        int far;
        if (sF.v != sG.v) far = (op == OP_MAX) ? (sF.v < sG.v ? PICK_F : PICK_G) : (sF.v > sG.v ? PICK_F : PICK_G);
        else far = (b0 != PICK_NONE) ? b0 : PICK_F;
        H->s[0] = (far == PICK_F) ? sF : sG;
        if (sF.v != sG.v && b0 != PICK_NONE && b0 != far) {
            num y = nadd(P[0], ndiv(nsub(fF[0], fG[0]), nsub(sG, sF)));
            if (y.v < P[0].v)
                push_pt(H, y, opval(op, pwl_eval(F, y), pwl_eval(G, y)), b0 == PICK_F ? sF : sG);
        }
    }
    for (int k = 0; k < K; k++) {
        num val = opval(op, fF[k], fG[k]);
        int last = (k == K - 1);
        num sF = last ? F->s[mF] : F->s[iF[k]];
        num sG = last ? G->s[mG] : G->s[iG[k]];
        if (!last) {
            int b0 = better(op, d[k]), b1 = better(op, d[k + 1]);
            if (sF.v != sG.v && b0 != PICK_NONE && b1 != PICK_NONE && b0 != b1) {
                num y = nadd(P[k], ndiv(nsub(fF[k], fG[k]), nsub(sG, sF)));
                if (y.v <= P[k].v) {
                    push_pt(H, P[k], val, b1 == PICK_F ? sF : sG);
                } else if (y.v >= P[k + 1].v) {
                    push_pt(H, P[k], val, b0 == PICK_F ? sF : sG);
                } else {
                    push_pt(H, P[k], val, b0 == PICK_F ? sF : sG);
                    push_pt(H, y, opval(op, pwl_eval(F, y), pwl_eval(G, y)), b1 == PICK_F ? sF : sG);
                }
            } else {
                int act = b0 != PICK_NONE ? b0 : b1;
                if (act == PICK_NONE) {
                    if (op == OP_MAX) act = (sG.v > sF.v) ? PICK_G : PICK_F;
                    else act = (sG.v < sF.v) ? PICK_G : PICK_F;
                }
                push_pt(H, P[k], val, act == PICK_F ? sF : sG);
            }
        } else {
            /* right tail */
            int bl = better(op, d[k]);
            int far;
            if (sF.v != sG.v) far = (op == OP_MAX) ? (sF.v > sG.v ? PICK_F : PICK_G) : (sF.v < sG.v ? PICK_F : PICK_G);
            else far = (bl != PICK_NONE) ? bl : PICK_F;
            if (sF.v != sG.v && bl != PICK_NONE && bl != far) {
                num y = nadd(P[k], ndiv(nsub(fF[k], fG[k]), nsub(sG, sF)));
                if (y.v > P[k].v) {
                    push_pt(H, P[k], val, bl == PICK_F ? sF : sG);
                    push_pt(H, y, opval(op, pwl_eval(F, y), pwl_eval(G, y)), far == PICK_F ? sF : sG);
                } else {
                    push_pt(H, P[k], val, far == PICK_F ? sF : sG);
                }
            } else {
                push_pt(H, P[k], val, far == PICK_F ? sF : sG);
            }
        }
    }
    free(P); free(iF); free(iG); free(fF); free(fG); free(d);
    pwl_canon(H);
}

/* SCALE(F, rho): the discounted function w_t / r = rho * w_t (Section 3):
 * values and slopes times rho, points unchanged; then CANON. */
static void pwl_scale(pwl *f, num rho)
{
    for (int j = 0; j < f->m; j++) f->v[j] = nmul(f->v[j], rho);
    for (int j = 0; j <= f->m; j++) f->s[j] = nmul(f->s[j], rho);
    pwl_canon(f);
}

/*
 * CLIP(F, a, b): restriction of the slopes of a convex function to [a, b]
 * with a = -S^a_t, b = -S^b_t (Section 3: the seller's v_t).  For convex F
 * the largest minorant with slopes in [a, b] is F with every slope clamped
 * into [a, b]: clamp, then CANON.  When a == b (no cost at t = 0) the result
 * is the line of slope a through the point where the slope of F passes a,
 * i.e. through x[q], q = clamp(i0 - 1, 0, m - 1), i0 = min{j : s[j] >= a}.
 */
static void pwl_clip(const pwl *F, num a, num b, pwl *V)
{
    int m = F->m;
    if (a.v == b.v) {
        int i0 = 0;
        while (i0 <= m && F->s[i0].v < a.v) i0++;
        int q = i0 - 1;
        if (q < 0) q = 0;
        if (q > m - 1) q = m - 1;
        pwl_vee(V, F->x[q], F->v[q], a, a);
        return;
    }
    pwl_copy(V, F);
    for (int j = 0; j <= m; j++) {
        if (V->s[j].v < a.v) V->s[j] = a;
        else if (V->s[j].v > b.v) V->s[j] = b;
    }
    pwl_canon(V);
}

/* mirror(F)(y) = F(-y). */
static void pwl_mirror(const pwl *F, pwl *R)
{
    int m = F->m;
    pwl_reserve(R, m);
    R->m = m;
    for (int j = 0; j < m; j++) { R->x[j] = nneg(F->x[m - 1 - j]); R->v[j] = F->v[m - 1 - j]; }
    for (int j = 0; j <= m; j++) R->s[j] = nneg(F->s[m - j]);
}

/*
 * A(y) = a*y + min_{y' >= y} (F(y') - a*y'): the cheapest position reachable
 * by buying stock at S^a (the "slope >= a" half of the rebalancing
 * restriction).  With h_j = v_j - a x_j and SM_j = min_{i > j} h_i (anchor
 * Q_j = the smallest i > j attaining it), on the piece (x_j, x_j+1)
 * A = min(F, L_j), L_j(y) = v_Q + a (y - x_Q), because the minimum of h over
 * [y, oo) is either h(y) on the piece or a breakpoint value to the right.
 * Each piece is of one of three kinds:
 *   FOLLOW  Q_j = j+1 and s_j+1 >= a: F itself (it touches L_j at x_j+1);
 *   SPLIT   Q_j > j+1, h_j < SM_j, s_j+1 > a and the crossing
 *           y = x_j + (SM_j - h_j)/(s_j+1 - a) lies strictly inside: F up to
 *           y, then L_j; the point y takes the value v_Q + a (y - x_Q); a y
 *           that rounds onto or past x_j+1 makes the piece FOLLOW;
 *   FLAT    otherwise: L_j.
 * The left tail is flat (slope a), the right tail is F (slope s_m > a).
 * Output: every x_j with value v_j and, after it, the SPLIT point of its
 * piece; each point carries the slope of the piece to its right; then CANON
 * (a point whose value would differ from v_j lies between two flat pieces
 * with one anchor and is dropped).  Requires s_0 < a < s_m.
 */
enum { PIECE_FLAT = 0, PIECE_FOLLOW = 1, PIECE_SPLIT = 2 };

static void env_scan_a(const pwl *F, num a, pwl *A)
{
    int m = F->m;
    num *h = (num *)malloc(sizeof(num) * m);
    double *SM = (double *)malloc(sizeof(double) * (m + 1));
    int *Q = (int *)malloc(sizeof(int) * (m + 1));
    for (int j = 0; j < m; j++) h[j] = nsub(F->v[j], nmul(a, F->x[j]));
    /* suffix minima strictly right of j, for j = m-2 down to 0 */
    for (int j = m - 2; j >= 0; j--) {
        if (j == m - 2 || h[j + 1].v <= SM[j + 1]) { SM[j] = h[j + 1].v; Q[j] = j + 1; }
        else { SM[j] = SM[j + 1]; Q[j] = Q[j + 1]; }
    }
    A->m = 0;
    pwl_reserve(A, 2 * m);
    A->s[0] = a;
    for (int j = 0; j < m; j++) {
        int kind = PIECE_FLAT;
        num y = nc(0.0);
        if (j < m - 1) {
            num sp = F->s[j + 1];
            if (Q[j] == j + 1) {
                if (sp.v >= a.v) kind = PIECE_FOLLOW;
            } else if (h[j].v < SM[j] && sp.v > a.v) {
                y = nadd(F->x[j], ndiv(nsub(h[Q[j]], h[j]), nsub(sp, a)));
                if (!(y.v < F->x[j + 1].v)) kind = PIECE_FOLLOW;
                else if (y.v > F->x[j].v) kind = PIECE_SPLIT;
            }
        }
        num sr = (j == m - 1) ? F->s[m] : (kind != PIECE_FLAT ? F->s[j + 1] : a);
        push_pt(A, F->x[j], F->v[j], sr);
        if (kind == PIECE_SPLIT) {
            int q = Q[j];
            push_pt(A, y, nadd(F->v[q], nmul(a, nsub(y, F->x[q]))), a);
        }
    }
    free(h); free(SM); free(Q);
    pwl_canon(A);
}

/*
 * ENV(F, a, b): the buyer's v_t (Section 3), the largest function below F
 * whose slopes lie in [a, b], i.e. v(y) = inf_delta F(y + delta)
 * + S^a delta^+ - S^b delta^-  (rebalancing at the ask/bid stock prices).
 * It is min(A, B) with A as in env_scan_a and B(y) = b*y + min_{y' <= y}
 * (F(y') - b*y') = mirror(A built on mirror(F) with slope -b), the
 * "slope <= b" half (stock sold at S^b).
 * When a == b the result is the line a*y + min_j (v[j] - a*x[j]) anchored at
 * the first minimising point.
 */
static void pwl_env(const pwl *F, num a, num b, pwl *V)
{
    int m = F->m;
    if (a.v == b.v) {
        int js = 0;
        double best = 0.0;
        for (int j = 0; j < m; j++) {
            double h = (nsub(F->v[j], nmul(a, F->x[j]))).v;
            if (j == 0 || h < best) { best = h; js = j; }
        }
        pwl_vee(V, F->x[js], F->v[js], a, a);
        return;
    }
    pwl A = {0}, B = {0}, R = {0}, RB = {0};
    env_scan_a(F, a, &A);
    pwl_mirror(F, &R);
    env_scan_a(&R, nneg(b), &RB);
    pwl_mirror(&RB, &B);
    pwl_canon(&B);
    pwl_merge(&A, &B, OP_MIN, V);
    pwl_free(&A); pwl_free(&B); pwl_free(&R); pwl_free(&RB);
}

/* ------------------------------------------------------------------------ */
/* Model (Section 4.1): u = exp(sigma sqrt(T/N)), d = 1/u, r = exp(R T/N),   */
/* S at node (t, c) = S0 u^(2c - t) by binary powering, costs k at t >= 1    */
/* and none at t = 0.                                                        */
/* ------------------------------------------------------------------------ */

/* e^x as the binary64 number nearest to the real number e^x: the model's u
 * and r are exponentials, and as binary64 numbers they are taken to be their
 * correctly rounded values.  Summed in binary128 (113-bit significand): the
 * argument is halved until |t| <= 1/16, the Taylor series of e^t is added
 * term by term up to t^30/30!, and the sum is squared back as often; the
 * binary128 result is within about 2^-100 (relative) of e^x for |x| <= 700,
 * and it is rounded once to binary64.  Pinned against decimal arithmetic at
 * 60 digits (tests/test_oracle_pins.py). */
static double exp_nearest(double x)
{
    __float128 t = x, term = 1, sum = 1;
    int s = 0;
    while (t > (__float128)0.0625 || t < -(__float128)0.0625) { t = t / 2; s++; }
    for (int n = 1; n <= 30; n++) { term = term * t / n; sum = sum + term; }
    while (s-- > 0) sum = sum * sum;
    return (double)sum;
}
enum { PAY_PUT = 0, PAY_CALL = 1, PAY_BULL = 2, PAY_PUT_CASH = 3, PAY_CALL_CASH = 4, PAY_BEAR = 5,
       PAY_STRADDLE = 6 };
enum { FL_EUROPEAN = 1u, FL_COST_AT_T0 = 2u };

/* base^n by binary powering: acc *= base^(2^i) for each set bit i, in
 * increasing i. */
static num upow(num base, int n)
{
    num acc = nc(1.0), b = base;
    int first = 1;
    while (n > 0) {
        if (n & 1) { acc = first ? b : nmul(acc, b); first = 0; }
        n >>= 1;
        if (n) b = nmul(b, b);
    }
    return acc;
}

typedef struct {
    int N, payoff; unsigned flags;
    num S0, K, K2, k, u, d, rho, r;
    double p;        /* risk-neutral up probability, k = 0 recursion only */
    num *S;          /* S[j + N + 1] = stock price for lattice index j */
} model;

static num stock(const model *md, int j) { return md->S[j + md->N + 1]; }

/* Payoff (xi, zeta) at a node with stock price S (Section 3: the holder
 * who exercises receives xi in cash and zeta shares; settlement in cash or
 * by delivery).  Delivered physically: put (K, -1), call (-K, 1).  Settled
 * in cash (zeta = 0): bull spread (S-K)^+ - (S-K2)^+, put (K-S)^+, call
 * (S-K)^+, bear spread (K2-S)^+ - (K-S)^+, straddle |S-K|. */
static void payoff(const model *md, num S, num *xi, num *zeta)
{
    *zeta = nc(0.0);
    switch (md->payoff) {
    case PAY_PUT: *xi = md->K; *zeta = nc(-1.0); break;
    case PAY_CALL: *xi = nneg(md->K); *zeta = nc(1.0); break;
    case PAY_BULL: *xi = nsub(npos(nsub(S, md->K)), npos(nsub(S, md->K2))); break;
    case PAY_PUT_CASH: *xi = npos(nsub(md->K, S)); break;
    case PAY_CALL_CASH: *xi = npos(nsub(S, md->K)); break;
    case PAY_BEAR: *xi = nsub(npos(nsub(md->K2, S)), npos(nsub(md->K, S))); break;
    default: {
        num e = nsub(S, md->K);
        *xi = e.v > 0.0 ? e : nneg(e);
    }
    }
}

static int model_init(model *md, double S0, double K, double K2, double R, double sigma,
                      double T, double k, int N, int pay, unsigned flags)
{
    if (!(N >= 1 && N <= (1 << 24))) return -1;
    if (!(isfinite(S0) && isfinite(K) && isfinite(R) && isfinite(sigma) && isfinite(T) && isfinite(k))) return -1;
    if (!(S0 > 0.0 && K > 0.0 && sigma > 0.0 && T > 0.0 && k >= 0.0 && k < 1.0)) return -1;
    if (pay < 0 || pay > 6) return -1;
    if ((pay == PAY_BULL || pay == PAY_BEAR) && !(isfinite(K2) && K2 > K)) return -1;
    memset(md, 0, sizeof(*md));
    md->N = N; md->payoff = pay; md->flags = flags;
    md->S0 = nc(S0); md->K = nc(K); md->K2 = nc(K2); md->k = nc(k);
    double dt = T / (double)N;
    double sq = sqrt(dt);
    double lam = sigma * sq;
    if (!(lam <= 700.0) || !(R * dt <= 700.0 && R * dt >= -700.0)) return -1;
    md->u = nc(exp_nearest(lam));
    md->r = nc(exp_nearest(R * dt));
    /* tangents: 0 = S0, 1 = sigma, 2 = R, 3 = k */
    if (NT >= 4) {
        md->S0.d[0] = 1.0;
        md->u.d[1] = md->u.v * sq;
        md->r.d[2] = md->r.v * dt;
        md->k.d[3] = 1.0;
    }
    md->d = ndiv(nc(1.0), md->u);
    md->rho = ndiv(nc(1.0), md->r);
    if (!(md->d.v < md->r.v && md->r.v < md->u.v)) return -1;
    md->p = (md->r.v - md->d.v) / (md->u.v - md->d.v);
    md->S = (num *)malloc(sizeof(num) * (2 * N + 3));
    for (int j = -(N + 1); j <= N + 1; j++) {
        num f = j >= 0 ? upow(md->u, j) : upow(md->d, -j);
        md->S[j + N + 1] = nmul(md->S0, f);
    }
    return 0;
}

/* Zero-cost CRR price (Section 3 and Appendix): no extra level;
 * V_N = max(xi + zeta S, 0), V_t = max(xi + zeta S, rho (p V_up + (1-p) V_dn)). */
static double crr_price(const model *md)
{
    int N = md->N;
    double *V = (double *)malloc(sizeof(double) * (N + 1));
    double p = md->p, q = 1.0 - md->p, rho = md->rho.v;
    int euro = (md->flags & FL_EUROPEAN) != 0;
    for (int c = 0; c <= N; c++) {
        num xi, ze; num S = stock(md, 2 * c - N);
        payoff(md, S, &xi, &ze);
        double P = xi.v + ze.v * S.v;
        V[c] = P > 0.0 ? P : 0.0;
    }
    for (int t = N - 1; t >= 0; t--) {
        for (int c = 0; c <= t; c++) {
            double cont = rho * (p * V[c + 1] + q * V[c]);
            if (euro) { V[c] = cont; continue; }
            num xi, ze; num S = stock(md, 2 * c - t);
            payoff(md, S, &xi, &ze);
            double P = xi.v + ze.v * S.v;
            if (P < 0.0) P = 0.0;
            V[c] = P > cont ? P : cont;
        }
    }
    double r = V[0];
    free(V);
    return r;
}

/*
 * The seller's (side 0, ask) or buyer's (side 1, bid) recursion, Section 3:
 *   level N+1: z = liquidation value y^- S^a - y^+ S^b (payoff (0, 0));
 *   t = N..0:  w = max(z_up, z_down); v = restrict(rho w) to slopes in
 *              [-S^a_t, -S^b_t]; seller z = max(u_t, v), buyer z = min(u_t, v);
 *   ask = z_0(0), bid = -z_0(0).
 * Up child of (t, c) is (t+1, c+1).  European variant: z_t = v_t for t < N.
 */
/* The optimal stock holding at t = 0 (the hedge): with f = rho max(z_1(1),
 * z_1(0)) and the rebalancing cost from no shares to y, the root's
 * restriction is v_0(0) = min over y of g(y), g(y) = f(y) + S^a_0 y for
 * y >= 0 and f(y) + S^b_0 y for y < 0 (Section 3: the cheapest portfolio
 * from which the node's expense is covered).  g is piecewise linear with
 * kinks at f's breakpoints and at 0, so its minimum is attained there; the
 * hedge is the interval [lo, hi] of those candidates whose g is within
 * 1e-12 (relative, floor 1) of the smallest. */
static void root_hedge(const pwl *f, num Sa, num Sb, double *lo, double *hi)
{
    double gmin = INFINITY;
    for (int pass = 0; pass < 2; pass++) {
        int first = 1;
        for (int j = 0; j <= f->m; j++) {
            double y = j < f->m ? f->x[j].v : 0.0;
            double g = pwl_eval(f, nc(y)).v + (y >= 0.0 ? Sa.v * y : Sb.v * y);
            if (pass == 0) {
                if (g < gmin) gmin = g;
            } else if (g <= gmin + 1e-12 * fmax(1.0, fabs(gmin))) {
                if (first || y < *lo) *lo = y;
                if (first || y > *hi) *hi = y;
                first = 0;
            }
        }
    }
}

/* The exercise map of one party (exmap, (N+1)(N+2)/2 bytes, node (t, c) at
 * t(t+1)/2 + c): 1 where exercise attains the party's expense at zero stock
 * holding -- the seller's z_t is max(u_t, v_t), so u_t(0) >= v_t(0); the
 * buyer's is min(u_t, v_t), so u_t(0) <= v_t(0), both evaluated by EVAL --
 * and 0 elsewhere, and at every t < N of the European variant, where there
 * is no exercise (Section 3). */
static int side_price_h(const model *md, int side, num *root, int64_t *bp_total, int *bp_max, double *hedge,
                        unsigned char *exmap)
{
    int N = md->N;
    pwl *cur = (pwl *)calloc(N + 2, sizeof(pwl));
    pwl *nxt = (pwl *)calloc(N + 2, sizeof(pwl));
    pwl W = {0}, V = {0}, U = {0};
    int euro = (md->flags & FL_EUROPEAN) != 0;
    num one = nc(1.0);
    for (int c = 0; c <= N + 1; c++) {
        num S = stock(md, 2 * c - (N + 1));
        num Sa = nmul(nadd(one, md->k), S), Sb = nmul(nsub(one, md->k), S);
        pwl_vee(&cur[c], nc(0.0), nc(0.0), nneg(Sa), nneg(Sb));
    }
    int64_t tot = 0; int mx = 0;
    for (int t = N; t >= 0; t--) {
        num kt = (t >= 1 || (md->flags & FL_COST_AT_T0)) ? md->k : nc(0.0);
        for (int c = 0; c <= t; c++) {
            num S = stock(md, 2 * c - t);
            num a = nneg(nmul(nadd(one, kt), S));
            num b = nneg(nmul(nsub(one, kt), S));
            pwl_merge(&cur[c + 1], &cur[c], OP_MAX, &W);
            pwl_scale(&W, md->rho);
            if (t == 0 && hedge) root_hedge(&W, nneg(a), nneg(b), &hedge[0], &hedge[1]);
            if (side == 0) pwl_clip(&W, a, b, &V);
            else pwl_env(&W, a, b, &V);
            if (euro && t < N) {
                pwl_swap(&nxt[c], &V);
            } else {
                num xi, ze;
                payoff(md, S, &xi, &ze);
                if (side == 0) pwl_vee(&U, ze, xi, a, b);
                else pwl_vee(&U, nneg(ze), nneg(xi), a, b);
                pwl_merge(&U, &V, side == 0 ? OP_MAX : OP_MIN, &nxt[c]);
            }
            if (exmap) {
                unsigned char e = 0;
                if (!(euro && t < N)) {
                    double v0 = pwl_eval(&V, nc(0.0)).v, u0 = pwl_eval(&U, nc(0.0)).v;
                    e = side == 0 ? (u0 >= v0) : (u0 <= v0);
                }
                exmap[(int64_t)t * (t + 1) / 2 + c] = e;
            }
            int bp = pwl_bp(&nxt[c]);
            tot += bp;
            if (bp > mx) mx = bp;
        }
        pwl *tmp = cur; cur = nxt; nxt = tmp;
    }
    *root = pwl_eval(&cur[0], nc(0.0));
    *bp_total = tot;
    *bp_max = mx;
    for (int c = 0; c <= N + 1; c++) { pwl_free(&cur[c]); pwl_free(&nxt[c]); }
    free(cur); free(nxt);
    pwl_free(&W); pwl_free(&V); pwl_free(&U);
    return 0;
}

static int side_price(const model *md, int side, num *root, int64_t *bp_total, int *bp_max)
{
    return side_price_h(md, side, root, bp_total, bp_max, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Exported API (ctypes).                                                    */
/* ------------------------------------------------------------------------ */

/* Prices one option.  out[0..2] = ask, bid, k = 0 price.  cnt[0..3] =
 * breakpoint total (ask side), total (bid side), max (ask), max (bid), over
 * levels 0..N.  grad (NT = 4 build only, may be NULL): grad[0..3] = d ask /
 * d(S0, sigma, R, k), grad[4..7] = d bid / d(...).  sides: bit 0 = ask,
 * bit 1 = bid.  Returns 0, or -1 for invalid parameters. */
int API(oracle_price)(double S0, double K, double K2, double R, double sigma, double T, double k,
                      int N, int pay, unsigned flags, int sides, double *out, int64_t *cnt, double *grad)
{
    model md;
    if (model_init(&md, S0, K, K2, R, sigma, T, k, N, pay, flags) != 0) return -1;
    out[0] = out[1] = NAN;
    cnt[0] = cnt[1] = 0; cnt[2] = cnt[3] = 0;
    if (grad) for (int i = 0; i < 8; i++) grad[i] = NAN;
    for (int side = 0; side < 2; side++) {
        if (!(sides & (1 << side))) continue;
        num root; int64_t tot; int mx;
        side_price(&md, side, &root, &tot, &mx);
        num price = side == 0 ? root : nneg(root);
        out[side] = price.v;
        cnt[side] = tot; cnt[2 + side] = mx;
        if (grad) for (int i = 0; i < NT && i < 4; i++) grad[4 * side + i] = price.d[i];
    }
    out[2] = crr_price(&md);
    free(md.S);
    return 0;
}

/* The hedges at t = 0 (root_hedge): out[0..1] = the seller's interval,
 * out[2..3] = the buyer's.  Returns 0, or -1 for invalid parameters. */
int API(oracle_hedge)(double S0, double K, double K2, double R, double sigma, double T, double k,
                      int N, int pay, unsigned flags, double *out)
{
    model md;
    if (model_init(&md, S0, K, K2, R, sigma, T, k, N, pay, flags) != 0) return -1;
    for (int side = 0; side < 2; side++) {
        num root; int64_t tot; int mx;
        side_price_h(&md, side, &root, &tot, &mx, out + 2 * side, NULL);
    }
    free(md.S);
    return 0;
}

/* The exercise maps of both parties (side_price_h): map[0 .. P-1] the
 * seller's, map[P .. 2P-1] the buyer's, P = (N+1)(N+2)/2.  Returns 0, or -1
 * for invalid parameters. */
int API(oracle_exercise)(double S0, double K, double K2, double R, double sigma, double T, double k,
                         int N, int pay, unsigned flags, unsigned char *map)
{
    model md;
    if (model_init(&md, S0, K, K2, R, sigma, T, k, N, pay, flags) != 0) return -1;
    const int64_t P = (int64_t)(N + 1) * (N + 2) / 2;
    for (int side = 0; side < 2; side++) {
        num root; int64_t tot; int mx;
        side_price_h(&md, side, &root, &tot, &mx, NULL, map + side * P);
    }
    free(md.S);
    return 0;
}

/* Stock price table S0 u^j, j = -(N+1)..N+1 (2N+3 entries), and the model
 * constants u, d, r, rho, p. */
int API(oracle_model)(double S0, double sigma, double R, double T, int N, double *table, double *consts)
{
    model md;
    if (model_init(&md, S0, 100.0, 200.0, R, sigma, T, 0.0, N, PAY_PUT, 0) != 0) return -1;
    for (int i = 0; i < 2 * N + 3; i++) table[i] = md.S[i].v;
    consts[0] = md.u.v; consts[1] = md.d.v; consts[2] = md.r.v; consts[3] = md.rho.v; consts[4] = md.p;
    free(md.S);
    return 0;
}

/* Binary64 operations counted on this thread since the previous call. */
uint64_t API(oracle_flops)(void)
{
    uint64_t f = g_flops;
    g_flops = 0;
    return f;
}

/* Single PWL operations for unit tests.  Functions travel as (m, x[m], v[m],
 * s[m+1]); the output arrays need room for the documented bound and *mo
 * receives the point count.  op: 0 = MERGE max, 1 = MERGE min, 2 = SCALE by
 * a, 3 = CLIP to [a, b], 4 = ENV to [a, b], 5 = CANON, 6 = ENV's buying half
 * A (slope >= a), 7 = ENV's selling half B (slope <= b).  Values only. */
static void load(pwl *f, int m, const double *x, const double *v, const double *s)
{
    pwl_reserve(f, m);
    f->m = m;
    for (int j = 0; j < m; j++) { f->x[j] = nc(x[j]); f->v[j] = nc(v[j]); }
    for (int j = 0; j <= m; j++) f->s[j] = nc(s[j]);
}

int API(oracle_pwl_op)(int op, int mF, const double *xF, const double *vF, const double *sF,
                       int mG, const double *xG, const double *vG, const double *sG,
                       double a, double b, int cap, int *mo, double *xo, double *vo, double *so)
{
    pwl F = {0}, G = {0}, H = {0};
    load(&F, mF, xF, vF, sF);
    if (op <= 1) { load(&G, mG, xG, vG, sG); pwl_merge(&F, &G, op, &H); }
    else if (op == 2) { pwl_copy(&H, &F); pwl_scale(&H, nc(a)); }
    else if (op == 3) pwl_clip(&F, nc(a), nc(b), &H);
    else if (op == 4) pwl_env(&F, nc(a), nc(b), &H);
    else if (op == 6) env_scan_a(&F, nc(a), &H);
    else if (op == 7) {   /* the "slope <= b" half: mirror(A(mirror F, -b)) */
        pwl R = {0}, RB = {0};
        pwl_mirror(&F, &R);
        env_scan_a(&R, nc(-b), &RB);
        pwl_mirror(&RB, &H);
        pwl_canon(&H);
        pwl_free(&R); pwl_free(&RB);
    }
    else { pwl_copy(&H, &F); pwl_canon(&H); }
    int rc = 0;
    if (H.m > cap) rc = -2;
    else {
        for (int j = 0; j < H.m; j++) { xo[j] = H.x[j].v; vo[j] = H.v[j].v; }
        for (int j = 0; j <= H.m; j++) so[j] = H.s[j].v;
    }
    *mo = H.m;
    pwl_free(&F); pwl_free(&G); pwl_free(&H);
    return rc;
}

/* EVAL for unit tests. */
double API(oracle_pwl_eval)(int m, const double *x, const double *v, const double *s, double y)
{
    pwl F = {0};
    load(&F, m, x, v, s);
    double r = pwl_eval(&F, nc(y)).v;
    pwl_free(&F);
    return r;
}

/* One node update for unit tests (the worked example of Section 3): children
 * zu, zd, node stock S, cost k_t, discount rho, exercise payoff (xi, zeta),
 * side 0 = seller, 1 = buyer.  Writes z and v. */
int API(oracle_node)(int side, int mu, const double *xu, const double *vu, const double *su,
                     int md_, const double *xd, const double *vd, const double *sd,
                     double S, double kt, double rho, double xi, double zeta, int cap,
                     int *mz, double *xz, double *vz, double *sz,
                     int *mv, double *xv, double *vv, double *sv)
{
    pwl Zu = {0}, Zd = {0}, W = {0}, V = {0}, U = {0}, Z = {0};
    load(&Zu, mu, xu, vu, su);
    load(&Zd, md_, xd, vd, sd);
    num one = nc(1.0);
    num a = nneg(nmul(nadd(one, nc(kt)), nc(S)));
    num b = nneg(nmul(nsub(one, nc(kt)), nc(S)));
    pwl_merge(&Zu, &Zd, OP_MAX, &W);
    pwl_scale(&W, nc(rho));
    if (side == 0) pwl_clip(&W, a, b, &V); else pwl_env(&W, a, b, &V);
    if (side == 0) pwl_vee(&U, nc(zeta), nc(xi), a, b);
    else pwl_vee(&U, nc(-zeta), nc(-xi), a, b);
    pwl_merge(&U, &V, side == 0 ? OP_MAX : OP_MIN, &Z);
    int rc = 0;
    if (Z.m > cap || V.m > cap) rc = -2;
    else {
        for (int j = 0; j < Z.m; j++) { xz[j] = Z.x[j].v; vz[j] = Z.v[j].v; }
        for (int j = 0; j <= Z.m; j++) sz[j] = Z.s[j].v;
        for (int j = 0; j < V.m; j++) { xv[j] = V.x[j].v; vv[j] = V.v[j].v; }
        for (int j = 0; j <= V.m; j++) sv[j] = V.s[j].v;
    }
    *mz = Z.m; *mv = V.m;
    pwl_free(&Zu); pwl_free(&Zd); pwl_free(&W); pwl_free(&V); pwl_free(&U); pwl_free(&Z);
    return rc;
}
