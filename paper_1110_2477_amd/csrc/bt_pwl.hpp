// bt_pwl.hpp -- piecewise-linear (PWL) expense functions on gfx950.
//
// The seller's and buyer's recursions of Zhang, Roux & Zastawniak (2011),
// Section 3, act on continuous PWL functions of the stock holding y.  A
// function is stored as m >= 1 strictly increasing points x[j] with values
// v[j], and m+1 slopes: s[0] left of x[0], s[j] on (x[j-1], x[j]), s[m]
// right of x[m-1].  Slopes are carried through every operation, never
// recomputed from points; a line is one anchor point with s[0] == s[1].
//
// Every operation below has one fixed sequence of IEEE binary64 operations
// (built with -ffp-contract=off), so a node's result does not depend on how
// the tree is mapped onto lanes, waves or workgroups:
//   EVAL   f(y) = v[i-1] + s[i](y - x[i-1]) with i = #{x[j] <= y}, or
//          v[0] + s[0](y - x[0]) when i = 0.
//   CANON  drop every point whose two adjacent slopes are equal; a function
//          left with no point keeps its first point as a line anchor.
//   MERGE  pointwise max or min (Section 3: w_t, and z_t = max/min(u_t, v_t)).
//   SCALE  the discount w_t / r, as multiplication by rho = 1/r.
//   CLIP   restriction of a convex function's slopes to [-S^a_t, -S^b_t].
//   ENV    the same restriction for a general function: the largest
//          minorant with slopes in [a, b], the cheapest rebalancing at the
//          ask/bid stock prices, built from a right-to-left sweep (stock
//          bought at S^a) and a mirrored sweep (stock sold at S^b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifdef BT_HOST_DEBUG
#define BTD __host__ __device__ inline
#else
#define BTD __device__ __forceinline__
#endif

namespace bt {

// Read view of a PWL function stored with an element stride.
struct View {
    const double *x, *v, *s;
    int m, st;
    BTD double X(int j) const { return x[(int64_t)j * st]; }
    BTD double V(int j) const { return v[(int64_t)j * st]; }
    BTD double S(int j) const { return s[(int64_t)j * st]; }
};

// Writable storage with room for `cap` points (and cap + 1 slopes).
struct Arr {
    double *x, *v, *s;
    int st, cap;
    BTD double &X(int j) const { return x[(int64_t)j * st]; }
    BTD double &V(int j) const { return v[(int64_t)j * st]; }
    BTD double &S(int j) const { return s[(int64_t)j * st]; }
    BTD View view(int m) const { return View{x, v, s, m, st}; }
};

enum { OPMAX = 0, OPMIN = 1 };
enum { PNONE = -1, PF = 0, PG = 1 };

BTD double eval_at(const View &f, int i, double y)
{
    if (i == 0) return f.V(0) + f.S(0) * (y - f.X(0));
    return f.V(i - 1) + f.S(i) * (y - f.X(i - 1));
}

BTD double eval(const View &f, double y)
{
    int lo = 0, hi = f.m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (f.X(mid) <= y) lo = mid + 1; else hi = mid;
    }
    return eval_at(f, lo, y);
}

template <int OP> BTD int better(double d)
{
    if (OP == OPMAX) return d > 0.0 ? PF : (d < 0.0 ? PG : PNONE);
    return d < 0.0 ? PF : (d > 0.0 ? PG : PNONE);
}

template <int OP> BTD double pick(double a, double b)
{
    if (OP == OPMAX) return a >= b ? a : b;
    return a <= b ? a : b;
}

// Output stream with CANON applied on the fly: a point is stored only if
// the slope arriving from its left differs from the slope leaving to its
// right.  Because a dropped point has equal slopes on both sides, the slope
// arriving at the next point is unchanged by the drop.
struct Emit {
    Arr o;
    int m;
    bool ovf, have0;
    double cur, x0, v0;
    BTD void start(const Arr &out, double s_left)
    {
        o = out; m = 0; ovf = false; have0 = false;
        cur = s_left;
        o.S(0) = s_left;
    }
    BTD void push(double x, double v, double s_right)
    {
        if (!have0) { x0 = x; v0 = v; have0 = true; }
        if (cur != s_right) {
            if (m < o.cap) { o.X(m) = x; o.V(m) = v; o.S(m + 1) = s_right; }
            else ovf = true;
            m++;
            cur = s_right;
        }
    }
    // Returns the point count, or -1 when the storage was too small.
    BTD int finish()
    {
        if (ovf) return -1;
        if (m == 0) { o.X(0) = x0; o.V(0) = v0; o.S(1) = o.S(0); m = 1; }
        return m;
    }
};

// In-place CANON of a stored function; returns the new point count.
BTD int canon(const Arr &f, int m)
{
    double s0 = f.S(0);
    int k = 0;
    for (int j = 0; j < m; j++) {
        // Writes go to indices k <= j (slopes k + 1 <= j + 1, equal only
        // when nothing was dropped, rewriting the same value), so s[j] and
        // s[j+1] still hold the input here.
        double sl = f.S(j), sr = f.S(j + 1);
        if (sl != sr) {
            double xj = f.X(j), vj = f.V(j);
            f.X(k) = xj; f.V(k) = vj; f.S(k + 1) = sr;
            k++;
        }
    }
    f.S(0) = s0;
    if (k == 0) { f.S(1) = s0; k = 1; }
    return k;
}

// MERGE(F, G, op) into `out`; returns the point count or -1 on overflow.
//  - P is the sorted union of both breakpoint lists (exact duplicates
//    merged); at every P_k, d_k = EVAL(F, P_k) - EVAL(G, P_k).
//  - Interval (P_k, P_k+1) with slopes sF != sG and d_k, d_k+1 of strictly
//    opposite signs crosses at y* = P_k + d_k / (sG - sF); y* <= P_k or
//    y* >= P_k+1 leaves the whole interval to the winner at the other end.
//    Without a crossing the winner is the better function at P_k, else at
//    P_k+1, else the one with the larger (MAX) / smaller (MIN) slope, F on a
//    full tie.
//  - Each tail's far winner follows from the slopes (MAX: smaller slope to
//    the left, larger to the right; MIN reversed); equal slopes fall back to
//    the sign of d at the end point, then F.  When the end point's winner
//    differs, the crossing y* = P_ref + d_ref / (sG - sF) is added if it lies
//    strictly outside the end point.
//  - Values are op(EVAL(F, y), EVAL(G, y)); slopes are the winner's.
// What MERGE emits for one union point P_k: the slope leaving P_k to the
// right (rs) and, when the interval after P_k holds a crossing, that point
// (cy, cv) and the slope leaving it (crs).
struct Slot {
    double rs;
    bool hc;
    double cy, cv, crs;
};

// Interval (P, P1) with F, G values fF, fG at P (d = fF - fG) and d1 at P1;
// iF, iG = #{points <= P} in F and G.
template <int OP>
BTD Slot slot_interval(const View &F, const View &G, double P, int iF, int iG, double fF, double fG,
                       double d, double P1, double d1)
{
    Slot o;
    o.hc = false; o.cy = 0.0; o.cv = 0.0; o.crs = 0.0;
    const double sF = F.S(iF), sG = G.S(iG);
    const int b0 = better<OP>(d), b1 = better<OP>(d1);
    if (sF != sG && b0 != PNONE && b1 != PNONE && b0 != b1) {
        const double y = P + (fF - fG) / (sG - sF);
        if (y <= P) {
            o.rs = b1 == PF ? sF : sG;
        } else if (y >= P1) {
            o.rs = b0 == PF ? sF : sG;
        } else {
            o.rs = b0 == PF ? sF : sG;
            o.hc = true;
            o.cy = y;
            o.cv = pick<OP>(eval_at(F, iF, y), eval_at(G, iG, y));
            o.crs = b1 == PF ? sF : sG;
        }
    } else {
        int act = b0 != PNONE ? b0 : b1;
        if (act == PNONE) {
            if (OP == OPMAX) act = (sG > sF) ? PG : PF;
            else act = (sG < sF) ? PG : PF;
        }
        o.rs = act == PF ? sF : sG;
    }
    return o;
}

// Right tail after the last union point P.
template <int OP>
BTD Slot slot_right(const View &F, const View &G, double P, double fF, double fG, double d)
{
    Slot o;
    o.hc = false; o.cy = 0.0; o.cv = 0.0; o.crs = 0.0;
    const double sF = F.S(F.m), sG = G.S(G.m);
    const int bl = better<OP>(d);
    int far;
    if (sF != sG) far = (OP == OPMAX) ? (sF > sG ? PF : PG) : (sF < sG ? PF : PG);
    else far = (bl != PNONE) ? bl : PF;
    if (sF != sG && bl != PNONE && bl != far) {
        const double y = P + (fF - fG) / (sG - sF);
        if (y > P) {
            o.rs = bl == PF ? sF : sG;
            o.hc = true;
            o.cy = y;
            o.cv = pick<OP>(eval_at(F, F.m, y), eval_at(G, G.m, y));
            o.crs = far == PF ? sF : sG;
        } else {
            o.rs = far == PF ? sF : sG;
        }
    } else {
        o.rs = far == PF ? sF : sG;
    }
    return o;
}

// Left tail before the first union point P0: the far-left slope s0 and an
// optional crossing (cy, cv) leaving with slope crs.
template <int OP>
BTD Slot slot_left(const View &F, const View &G, double P0, double fF, double fG, double d)
{
    Slot o;
    o.hc = false; o.cy = 0.0; o.cv = 0.0; o.crs = 0.0;
    const double sF = F.S(0), sG = G.S(0);
    const int b0 = better<OP>(d);
    int far;
    if (sF != sG) far = (OP == OPMAX) ? (sF < sG ? PF : PG) : (sF > sG ? PF : PG);
    else far = (b0 != PNONE) ? b0 : PF;
    o.rs = far == PF ? sF : sG;
    if (sF != sG && b0 != PNONE && b0 != far) {
        const double y = P0 + (fF - fG) / (sG - sF);
        if (y < P0) {
            o.hc = true;
            o.cy = y;
            o.cv = pick<OP>(eval_at(F, 0, y), eval_at(G, 0, y));
            o.crs = b0 == PF ? sF : sG;
        }
    }
    return o;
}

// MERGE(F, G, op) into `out`; returns the point count or -1 on overflow.
//  - P is the sorted union of both breakpoint lists (exact duplicates
//    merged); at every P_k, d_k = EVAL(F, P_k) - EVAL(G, P_k).
//  - Interval (P_k, P_k+1) with slopes sF != sG and d_k, d_k+1 of strictly
//    opposite signs crosses at y* = P_k + d_k / (sG - sF); y* <= P_k or
//    y* >= P_k+1 leaves the whole interval to the winner at the other end.
//    Without a crossing the winner is the better function at P_k, else at
//    P_k+1, else the one with the larger (MAX) / smaller (MIN) slope, F on a
//    full tie.
//  - Each tail's far winner follows from the slopes (MAX: smaller slope to
//    the left, larger to the right; MIN reversed); equal slopes fall back to
//    the sign of d at the end point, then F.  When the end point's winner
//    differs, the crossing y* = P_ref + d_ref / (sG - sF) is added if it lies
//    strictly outside the end point.
//  - Values are op(EVAL(F, y), EVAL(G, y)); slopes are the winner's.
template <int OP>
BTD int merge(const View &F, const View &G, const Arr &out)
{
    const double INF = __builtin_huge_val();
    int a = 0, b = 0;
    double P, fF, fG, d;
    int iF, iG;
    {
        const double xa = F.X(0), xb = G.X(0);
        if (xa < xb) { P = xa; a = 1; }
        else if (xb < xa) { P = xb; b = 1; }
        else { P = xa; a = 1; b = 1; }
        iF = a; iG = b;
        fF = eval_at(F, iF, P);
        fG = eval_at(G, iG, P);
        d = fF - fG;
    }
    Emit e;
    {
        const Slot L = slot_left<OP>(F, G, P, fF, fG, d);
        e.start(out, L.rs);
        if (L.hc) e.push(L.cy, L.cv, L.crs);
    }
    for (;;) {
        const double val = pick<OP>(fF, fG);
        if (a < F.m || b < G.m) {
            const double xa = a < F.m ? F.X(a) : INF, xb = b < G.m ? G.X(b) : INF;
            double P1;
            if (xa < xb) { P1 = xa; a++; }
            else if (xb < xa) { P1 = xb; b++; }
            else { P1 = xa; a++; b++; }
            const int iF1 = a, iG1 = b;
            const double fF1 = eval_at(F, iF1, P1), fG1 = eval_at(G, iG1, P1);
            const double d1 = fF1 - fG1;
            const Slot o = slot_interval<OP>(F, G, P, iF, iG, fF, fG, d, P1, d1);
            e.push(P, val, o.rs);
            if (o.hc) e.push(o.cy, o.cv, o.crs);
            P = P1; iF = iF1; iG = iG1; fF = fF1; fG = fG1; d = d1;
        } else {
            const Slot o = slot_right<OP>(F, G, P, fF, fG, d);
            e.push(P, val, o.rs);
            if (o.hc) e.push(o.cy, o.cv, o.crs);
            break;
        }
    }
    return e.finish();
}

// SCALE by rho in place, then CANON.
BTD int scale(const Arr &f, int m, double rho)
{
    for (int j = 0; j < m; j++) f.V(j) = f.V(j) * rho;
    for (int j = 0; j <= m; j++) f.S(j) = f.S(j) * rho;
    return canon(f, m);
}

// CLIP(F, a, b) in place (seller, F convex).  a < b: clamp every slope into
// [a, b], then CANON.  a == b: the line of slope a through x[q],
// q = clamp(i0 - 1, 0, m - 1), i0 = min{j : s[j] >= a}.
BTD int clip(const Arr &f, int m, double a, double b)
{
    if (a == b) {
        int i0 = 0;
        while (i0 <= m && f.S(i0) < a) i0++;
        int q = i0 - 1;
        if (q < 0) q = 0;
        if (q > m - 1) q = m - 1;
        double xq = f.X(q), vq = f.V(q);
        f.X(0) = xq; f.V(0) = vq; f.S(0) = a; f.S(1) = a;
        return 1;
    }
    for (int j = 0; j <= m; j++) {
        double s = f.S(j);
        if (s < a) f.S(j) = a;
        else if (s > b) f.S(j) = b;
    }
    return canon(f, m);
}

// Accessors of F or of its mirror image y -> -y.
template <bool MIR> struct Src {
    View f;
    BTD double X(int j) const { return MIR ? -f.X(f.m - 1 - j) : f.X(j); }
    BTD double V(int j) const { return MIR ? f.V(f.m - 1 - j) : f.V(j); }
    BTD double S(int j) const { return MIR ? -f.S(f.m - j) : f.S(j); }
};

// Reverse points [0, n) and slopes [0, n) in place.
BTD void reverse_pts(const Arr &o, int n)
{
    for (int i = 0, j = n - 1; i < j; i++, j--) {
        double t;
        t = o.X(i); o.X(i) = o.X(j); o.X(j) = t;
        t = o.V(i); o.V(i) = o.V(j); o.V(j) = t;
        t = o.S(i); o.S(i) = o.S(j); o.S(j) = t;
    }
}

// A(y) = a y + min_{y' >= y} (F(y') - a y') over F (or its mirror): the
// buying half of the restriction.  With h_j = v_j - a x_j, SM_j the minimum
// of h_i over i > j and Q_j the smallest such i attaining it, the piece
// (x_j, x_j+1) of A is min(F, L_j), L_j(y) = v_Q + a (y - x_Q), one of
//   FOLLOW  Q_j = j+1 and s_j+1 >= a, or a crossing that rounds onto or past
//           x_j+1: F;
//   SPLIT   Q_j > j+1, h_j < SM_j, s_j+1 > a and the crossing
//           y = x_j + (SM_j - h_j) / (s_j+1 - a) strictly inside: F, then L_j
//           from y (valued v_Q + a (y - x_Q));
//   FLAT    otherwise: L_j.
// Left tail flat (slope a), right tail F.  Points: every x_j with v_j and
// the SPLIT points, each with the slope to its right; then CANON.  Computed
// right to left with a running minimum (ties keep the nearer index), written
// in reverse and flipped.  Requires s_0 < a < s_m.  Returns the count or -1
// on overflow.
template <bool MIR>
BTD int sweep_a(const View &F, double a, const Arr &o)
{
    Src<MIR> f{F};
    const int m = F.m;
    int n = 0;
    double SMc = 0.0, xq = 0.0, vq = 0.0;
    int Qc = -1;
    double xr = 0.0;  // x_{j+1}
    for (int j = m - 1; j >= 0; j--) {
        const double xj = f.X(j), vj = f.V(j);
        const double hj = vj - a * xj;
        double rs;
        if (j == m - 1) {
            rs = f.S(m);
        } else {
            const double sp = f.S(j + 1);
            int kind = 0;  // 0 FLAT, 1 FOLLOW, 2 SPLIT
            double y = 0.0;
            if (Qc == j + 1) {
                if (sp >= a) kind = 1;
            } else if (hj < SMc && sp > a) {
                y = xj + (SMc - hj) / (sp - a);
                if (!(y < xr)) kind = 1;
                else if (y > xj) kind = 2;
            }
            if (kind == 2) {
                if (n >= o.cap) return -1;
                o.X(n) = y; o.V(n) = vq + a * (y - xq); o.S(n) = a;
                n++;
            }
            rs = kind != 0 ? sp : a;
        }
        if (n >= o.cap) return -1;
        o.X(n) = xj; o.V(n) = vj; o.S(n) = rs;
        n++;
        if (j == m - 1 || hj <= SMc) { SMc = hj; Qc = j; xq = xj; vq = vj; }
        xr = xj;
    }
    reverse_pts(o, n);
    // s[i] now holds the right slope of point i: shift to s[i+1], left tail a
    for (int i = n - 1; i >= 0; i--) o.S(i + 1) = o.S(i);
    o.S(0) = a;
    return canon(o, n);
}

// Mirror in place: x_j <- -x_{n-1-j}, v_j <- v_{n-1-j}, s_j <- -s_{n-j}.
BTD void mirror_inplace(const Arr &o, int n)
{
    for (int i = 0, j = n - 1; i < j; i++, j--) {
        double t;
        t = o.X(i); o.X(i) = o.X(j); o.X(j) = t;
        t = o.V(i); o.V(i) = o.V(j); o.V(j) = t;
    }
    for (int i = 0; i < n; i++) o.X(i) = -o.X(i);
    for (int i = 0, j = n; i < j; i++, j--) {
        double t = o.S(i); o.S(i) = o.S(j); o.S(j) = t;
    }
    for (int i = 0; i <= n; i++) o.S(i) = -o.S(i);
}

}  // namespace bt
