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
//          ask/bid stock prices, built from a buying half (slopes >= a) and a
//          mirrored selling half (slopes <= b).
//
// The number type T is double, or D4: a value with its derivatives with
// respect to (S0, sigma, R, k) carried forward through every operation (the
// Greeks).  Decisions look at values only, so both types take the same
// branches and produce the same value bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// BT_HOST_BUILD (or BT_HOST_DEBUG, the CPU test builds) compiles every
// operation for the host as well: the host-thread baseline of Section 4.2
// runs the same node update as the kernels.
#if defined(BT_HOST_DEBUG) || defined(BT_HOST_BUILD)
#define BTD __host__ __device__ inline
#else
#define BTD __device__ __forceinline__
#endif

// Every View and Arr points into global memory (level buffers, workspace,
// pool, arena).  Accessing them through a global-qualified pointer lets the
// compiler emit global instead of flat loads and stores, which do not wait
// on LDS traffic.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(BT_HOST_DEBUG) && !defined(BT_HOST_BUILD)
#define BT_GLOBAL __attribute__((address_space(1)))
#else
#define BT_GLOBAL
#endif

namespace bt {

// A value and its four tangents (d/dS0, d/dsigma, d/dR, d/dk).
struct D4 {
    double v, d[4];
};

BTD D4 operator+(const D4 &a, const D4 &b)
{
    D4 r;
    r.v = a.v + b.v;
    for (int i = 0; i < 4; i++) r.d[i] = a.d[i] + b.d[i];
    return r;
}
BTD D4 operator-(const D4 &a, const D4 &b)
{
    D4 r;
    r.v = a.v - b.v;
    for (int i = 0; i < 4; i++) r.d[i] = a.d[i] - b.d[i];
    return r;
}
BTD D4 operator-(const D4 &a)
{
    D4 r;
    r.v = -a.v;
    for (int i = 0; i < 4; i++) r.d[i] = -a.d[i];
    return r;
}
BTD D4 operator*(const D4 &a, const D4 &b)
{
    D4 r;
    r.v = a.v * b.v;
    for (int i = 0; i < 4; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
BTD D4 operator/(const D4 &a, const D4 &b)
{
    D4 r;
    r.v = a.v / b.v;
    for (int i = 0; i < 4; i++) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}

BTD double val(double x) { return x; }
BTD double val(const D4 &x) { return x.v; }

template <typename T> BTD T mk(double x);
template <> BTD double mk<double>(double x) { return x; }
template <> BTD D4 mk<D4>(double x)
{
    D4 r;
    r.v = x;
    r.d[0] = r.d[1] = r.d[2] = r.d[3] = 0.0;
    return r;
}

// Read view of a PWL function stored with an element stride.
template <typename T>
struct View {
    const T *x, *v, *s;
    int m, st;
    BTD const T &X(int j) const { return ((const BT_GLOBAL T *)x)[(int64_t)j * st]; }
    BTD const T &V(int j) const { return ((const BT_GLOBAL T *)v)[(int64_t)j * st]; }
    BTD const T &S(int j) const { return ((const BT_GLOBAL T *)s)[(int64_t)j * st]; }
};

// Writable storage with room for `cap` points (and cap + 1 slopes).
template <typename T>
struct Arr {
    T *x, *v, *s;
    int st, cap;
    BTD T &X(int j) const { return ((BT_GLOBAL T *)x)[(int64_t)j * st]; }
    BTD T &V(int j) const { return ((BT_GLOBAL T *)v)[(int64_t)j * st]; }
    BTD T &S(int j) const { return ((BT_GLOBAL T *)s)[(int64_t)j * st]; }
    BTD View<T> view(int m) const { return View<T>{x, v, s, m, st}; }
};

enum { OPMAX = 0, OPMIN = 1 };
enum { PNONE = -1, PF = 0, PG = 1 };

// The piece of f holding abscissa y when i = #{points <= y}: the line
// through (x, v) with slope s (the left tail through the first point for
// i = 0).
template <typename T>
struct Seg {
    T x, v, s;
};

// One point with its two slopes, held in registers (a node's exercise
// function u_t); the accessors of View.
template <typename T>
struct Kink {
    T x, v, s0, s1;
    int m;
    BTD T X(int) const { return x; }
    BTD T V(int) const { return v; }
    BTD T S(int j) const { return j == 0 ? s0 : s1; }
};

template <typename T, typename F>
BTD Seg<T> seg_at(const F &f, int i)
{
    const int p = i > 0 ? i - 1 : 0;   // no branch: the loads issue together
    return Seg<T>{f.X(p), f.V(p), f.S(i)};
}

template <typename T>
BTD T seg_eval(const Seg<T> &g, const T &y)
{
    return g.v + g.s * (y - g.x);
}

template <typename T, typename F>
BTD T eval_at(const F &f, int i, const T &y)
{
    return seg_eval<T>(seg_at<T>(f, i), y);
}

template <typename T>
BTD T eval(const View<T> &f, const T &y)
{
    int lo = 0, hi = f.m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (val(f.X(mid)) <= val(y)) lo = mid + 1; else hi = mid;
    }
    return eval_at<T>(f, lo, y);
}

template <int OP> BTD int better(double d)
{
    if (OP == OPMAX) return d > 0.0 ? PF : (d < 0.0 ? PG : PNONE);
    return d < 0.0 ? PF : (d > 0.0 ? PG : PNONE);
}

// Whether pick<OP>(a, b) takes a.
template <int OP, typename T> BTD bool pick_first(const T &a, const T &b)
{
    return OP == OPMAX ? val(a) >= val(b) : val(a) <= val(b);
}

template <int OP, typename T> BTD T pick(const T &a, const T &b)
{
    if (OP == OPMAX) return val(a) >= val(b) ? a : b;
    return val(a) <= val(b) ? a : b;
}

// Output stream with CANON applied on the fly: a point is stored only if
// the slope arriving from its left differs from the slope leaving to its
// right.  Because a dropped point has equal slopes on both sides, the slope
// arriving at the next point is unchanged by the drop.
template <typename T>
struct Emit {
    Arr<T> o;
    int m;
    bool ovf, have0;
    double cur;
    T x0, v0;
    BTD void start(const Arr<T> &out, const T &s_left)
    {
        o = out; m = 0; ovf = false; have0 = false;
        cur = val(s_left);
        o.S(0) = s_left;
    }
    BTD void push(const T &x, const T &v, const T &s_right)
    {
        if (!have0) { x0 = x; v0 = v; have0 = true; }
        if (cur != val(s_right)) {
            if (m < o.cap) { o.X(m) = x; o.V(m) = v; o.S(m + 1) = s_right; }
            else ovf = true;
            m++;
            cur = val(s_right);
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

// Emit followed by SCALE by rho and its CANON, in one pass: a point that
// Emit keeps is stored with v rho and s rho unless its scaled slopes are
// equal (the scaled CANON's decision on Emit's sequence).  When nothing is
// stored, the one point left is Emit's (its first kept point, else the first
// pushed), as SCALE and CANON after Emit would leave it.
template <typename T>
struct EmitScaled {
    Arr<T> o;
    T rho;
    int m, mu;
    bool ovf, have0;
    double cur, curs;
    T x0, v0, xk, vk;
    BTD void start(const Arr<T> &out, const T &s_left)
    {
        o = out; m = 0; mu = 0; ovf = false; have0 = false;
        cur = val(s_left);
        const T ss = s_left * rho;
        curs = val(ss);
        o.S(0) = ss;
    }
    BTD void push(const T &x, const T &v, const T &s_right)
    {
        if (!have0) { x0 = x; v0 = v; have0 = true; }
        if (cur != val(s_right)) {
            if (mu == 0) { xk = x; vk = v; }
            if (mu >= o.cap) ovf = true;   // where Emit would overflow
            mu++;
            cur = val(s_right);
            const T ss = s_right * rho;
            if (curs != val(ss)) {
                if (m < o.cap) { o.X(m) = x; o.V(m) = v * rho; o.S(m + 1) = ss; }
                else ovf = true;
                m++;
                curs = val(ss);
            }
        }
    }
    BTD int finish()
    {
        if (ovf) return -1;
        if (m == 0) {
            if (mu == 0) { o.X(0) = x0; o.V(0) = v0 * rho; }
            else { o.X(0) = xk; o.V(0) = vk * rho; }
            o.S(1) = o.S(0);
            m = 1;
        }
        return m;
    }
};

// Points per group of the in-place loops below: a group's loads issue
// before its stores (a store may alias a later load, so the compiler would
// otherwise wait for each point's round trip to memory).
constexpr int PWL_GROUP = 4;
// Dual numbers take a point at a time: a group of them would spill.
template <typename T>
constexpr int pwl_group() { return sizeof(T) == sizeof(double) ? PWL_GROUP : 1; }

// In-place CANON of a stored function after mapping each value by fv and
// each slope by fs, in one pass; returns the new point count.
template <typename T, class FV, class FS>
BTD int canon_map(const Arr<T> &f, int m, FV fv, FS fs)
{
    constexpr int B = pwl_group<T>();
    const T s0 = fs(f.S(0));
    int k = 0;
    double sl = val(s0);
    for (int j0 = 0; j0 < m; j0 += B) {
        // Writes go to indices k <= j (slopes k + 1 <= j + 1, equal only
        // when nothing was dropped, rewriting the same value), so the group's
        // inputs, read first, are the original ones, and s[j] is the s[j+1]
        // read for the point before.
        T xs[B], vs[B], ss[B];
#pragma unroll
        for (int u = 0; u < B; u++) {
            if (j0 + u < m) { xs[u] = f.X(j0 + u); vs[u] = fv(f.V(j0 + u)); ss[u] = fs(f.S(j0 + u + 1)); }
        }
#pragma unroll
        for (int u = 0; u < B; u++) {
            if (j0 + u < m) {
                const double sr = val(ss[u]);
                if (sl != sr) {
                    f.X(k) = xs[u]; f.V(k) = vs[u]; f.S(k + 1) = ss[u];
                    k++;
                }
                sl = sr;
            }
        }
    }
    f.S(0) = s0;
    if (k == 0) { f.S(1) = s0; k = 1; }
    return k;
}

// In-place CANON of a stored function; returns the new point count.
template <typename T>
BTD int canon(const Arr<T> &f, int m)
{
    const auto same = [](const T &y) { return y; };
    return canon_map(f, m, same, same);
}

// What MERGE emits for one union point P_k: the slope leaving P_k to the
// right (rs) and, when the interval after P_k holds a crossing, that point
// (cy, cv) and the slope leaving it (crs).
// rsF, cvF, crsF: rs, cv and crs are F's (else G's), so that the same point
// can be rebuilt from the pieces (dual numbers take their decisions on the
// values first).
template <typename T>
struct Slot {
    T rs;
    bool hc;
    T cy, cv, crs;
    bool rsF, cvF, crsF;
};

// Interval (P, P1) with F, G values fF, fG at P and d1 = F - G at P1;
// gF, gG: the pieces of F and G over the interval (seg_at with
// #{points <= P}).
template <int OP, typename T>
BTD Slot<T> slot_interval_seg(const Seg<T> &gF, const Seg<T> &gG, const T &P, const T &fF, const T &fG,
                              const T &P1, double d1)
{
    Slot<T> o;
    o.hc = false;
    const T sF = gF.s, sG = gG.s;
    const int b0 = better<OP>(val(fF) - val(fG)), b1 = better<OP>(d1);
    o.cvF = o.crsF = false;
    if (val(sF) != val(sG) && b0 != PNONE && b1 != PNONE && b0 != b1) {
        const T y = P + (fF - fG) / (sG - sF);
        if (val(y) <= val(P)) {
            o.rsF = b1 == PF;
        } else if (val(y) >= val(P1)) {
            o.rsF = b0 == PF;
        } else {
            o.rsF = b0 == PF;
            o.hc = true;
            o.cy = y;
            const T eF = seg_eval<T>(gF, y), eG = seg_eval<T>(gG, y);
            o.cvF = pick_first<OP, T>(eF, eG);
            o.cv = o.cvF ? eF : eG;
            o.crsF = b1 == PF;
            o.crs = o.crsF ? sF : sG;
        }
    } else {
        int act = b0 != PNONE ? b0 : b1;
        if (act == PNONE) {
            if (OP == OPMAX) act = (val(sG) > val(sF)) ? PG : PF;
            else act = (val(sG) < val(sF)) ? PG : PF;
        }
        o.rsF = act == PF;
    }
    o.rs = o.rsF ? sF : sG;
    return o;
}

// iF, iG = #{points <= P} in F and G.
template <int OP, typename T, typename FF, typename GG>
BTD Slot<T> slot_interval(const FF &F, const GG &G, const T &P, int iF, int iG, const T &fF, const T &fG,
                          const T &P1, double d1)
{
    return slot_interval_seg<OP, T>(seg_at<T>(F, iF), seg_at<T>(G, iG), P, fF, fG, P1, d1);
}

// Right tail after the last union point P.
template <int OP, typename T, typename FF, typename GG>
BTD Slot<T> slot_right(const FF &F, const GG &G, const T &P, const T &fF, const T &fG)
{
    Slot<T> o;
    o.hc = false;
    const T sF = F.S(F.m), sG = G.S(G.m);
    const int bl = better<OP>(val(fF) - val(fG));
    int far;
    if (val(sF) != val(sG)) far = (OP == OPMAX) ? (val(sF) > val(sG) ? PF : PG) : (val(sF) < val(sG) ? PF : PG);
    else far = (bl != PNONE) ? bl : PF;
    o.cvF = o.crsF = false;
    if (val(sF) != val(sG) && bl != PNONE && bl != far) {
        const T y = P + (fF - fG) / (sG - sF);
        if (val(y) > val(P)) {
            o.rsF = bl == PF;
            o.hc = true;
            o.cy = y;
            const T eF = eval_at<T>(F, F.m, y), eG = eval_at<T>(G, G.m, y);
            o.cvF = pick_first<OP, T>(eF, eG);
            o.cv = o.cvF ? eF : eG;
            o.crsF = far == PF;
            o.crs = o.crsF ? sF : sG;
        } else {
            o.rsF = far == PF;
        }
    } else {
        o.rsF = far == PF;
    }
    o.rs = o.rsF ? sF : sG;
    return o;
}

// Left tail before the first union point P0: the far-left slope s0 (rs) and
// an optional crossing (cy, cv) leaving with slope crs.
template <int OP, typename T, typename FF, typename GG>
BTD Slot<T> slot_left(const FF &F, const GG &G, const T &P0, const T &fF, const T &fG)
{
    Slot<T> o;
    o.hc = false;
    const T sF = F.S(0), sG = G.S(0);
    const int b0 = better<OP>(val(fF) - val(fG));
    int far;
    if (val(sF) != val(sG)) far = (OP == OPMAX) ? (val(sF) < val(sG) ? PF : PG) : (val(sF) > val(sG) ? PF : PG);
    else far = (b0 != PNONE) ? b0 : PF;
    o.rs = far == PF ? sF : sG;
    if (val(sF) != val(sG) && b0 != PNONE && b0 != far) {
        const T y = P0 + (fF - fG) / (sG - sF);
        if (val(y) < val(P0)) {
            o.hc = true;
            o.cy = y;
            o.cv = pick<OP, T>(eval_at<T>(F, 0, y), eval_at<T>(G, 0, y));
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
// F and G are any types with m, X(j), V(j), S(j).
template <int OP, typename T, class EM, typename FF, typename GG>
BTD int merge_em(const FF &F, const GG &G, const Arr<T> &out, EM &e)
{
    const double INF = __builtin_huge_val();
    int a = 0, b = 0;
    T P, fF, fG;
    int iF, iG;
    // the pieces of F and G that hold P (seg_at(F, iF), seg_at(G, iG)),
    // carried from one union point to the next instead of loaded again
    Seg<T> gF, gG;
    {
        const double xa = val(F.X(0)), xb = val(G.X(0));
        if (xa < xb) { P = F.X(0); a = 1; }
        else if (xb < xa) { P = G.X(0); b = 1; }
        else { P = F.X(0); a = 1; b = 1; }
        iF = a; iG = b;
        gF = seg_at<T>(F, iF);
        gG = seg_at<T>(G, iG);
        fF = seg_eval<T>(gF, P);
        fG = seg_eval<T>(gG, P);
    }
    {
        const Slot<T> L = slot_left<OP, T>(F, G, P, fF, fG);
        e.start(out, L.rs);
        if (L.hc) e.push(L.cy, L.cv, L.crs);
    }
    for (;;) {
        const T vv = pick<OP, T>(fF, fG);
        if (a < F.m || b < G.m) {
            const double xa = a < F.m ? val(F.X(a)) : INF, xb = b < G.m ? val(G.X(b)) : INF;
            T P1;
            if (xa < xb) { P1 = F.X(a); a++; }
            else if (xb < xa) { P1 = G.X(b); b++; }
            else { P1 = F.X(a); a++; b++; }
            const int iF1 = a, iG1 = b;
            const Seg<T> gF1 = iF1 == iF ? gF : seg_at<T>(F, iF1);
            const Seg<T> gG1 = iG1 == iG ? gG : seg_at<T>(G, iG1);
            const T fF1 = seg_eval<T>(gF1, P1), fG1 = seg_eval<T>(gG1, P1);
            const Slot<T> o = slot_interval_seg<OP, T>(gF, gG, P, fF, fG, P1, val(fF1) - val(fG1));
            e.push(P, vv, o.rs);
            if (o.hc) e.push(o.cy, o.cv, o.crs);
            P = P1; iF = iF1; iG = iG1; fF = fF1; fG = fG1; gF = gF1; gG = gG1;
        } else {
            const Slot<T> o = slot_right<OP, T>(F, G, P, fF, fG);
            e.push(P, vv, o.rs);
            if (o.hc) e.push(o.cy, o.cv, o.crs);
            break;
        }
    }
    return e.finish();
}

template <int OP, typename T, typename FF, typename GG>
BTD int merge(const FF &F, const GG &G, const Arr<T> &out)
{
    Emit<T> e;
    return merge_em<OP, T>(F, G, out, e);
}

// MERGE, then SCALE by rho with its CANON, in one pass over the output.
template <int OP, typename T, typename FF, typename GG>
BTD int merge_scale(const FF &F, const GG &G, const Arr<T> &out, const T &rho)
{
    EmitScaled<T> e;
    e.rho = rho;
    return merge_em<OP, T>(F, G, out, e);
}

// SCALE by rho in place, then CANON (one pass).
template <typename T>
BTD int scale(const Arr<T> &f, int m, const T &rho)
{
    const auto mul = [rho](const T &y) { return y * rho; };
    return canon_map(f, m, mul, mul);
}

// CLIP(F, a, b) in place (seller, F convex).  a < b: clamp every slope into
// [a, b], then CANON.  a == b: the line of slope a through x[q],
// q = clamp(i0 - 1, 0, m - 1), i0 = min{j : s[j] >= a}.
template <typename T>
BTD int clip(const Arr<T> &f, int m, const T &a, const T &b)
{
    if (val(a) == val(b)) {
        int i0 = 0;
        while (i0 <= m && val(f.S(i0)) < val(a)) i0++;
        int q = i0 - 1;
        if (q < 0) q = 0;
        if (q > m - 1) q = m - 1;
        const T xq = f.X(q), vq = f.V(q);
        f.X(0) = xq; f.V(0) = vq; f.S(0) = a; f.S(1) = a;
        return 1;
    }
    // the clamp and CANON in one pass
    const auto same = [](const T &y) { return y; };
    const auto clamp = [a, b](const T &sl) { return val(sl) < val(a) ? a : (val(sl) > val(b) ? b : sl); };
    return canon_map(f, m, same, clamp);
}

// Accessors of F or of its mirror image y -> -y.
template <bool MIR, typename T>
struct Src {
    View<T> f;
    int m;
    BTD T X(int j) const { return MIR ? -f.X(f.m - 1 - j) : f.X(j); }
    BTD T V(int j) const { return MIR ? f.V(f.m - 1 - j) : f.V(j); }
    BTD T S(int j) const { return MIR ? -f.S(f.m - j) : f.S(j); }
};

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
// right to left with a running minimum (ties keep the nearer index):
// sweep_raw leaves the points in `o` in that order (decreasing x), each with
// its right slope at the same index, and returns their count (-1 on
// overflow); sweep_a reads them back in increasing x into `o2` (not the raw
// array) with CANON in the same pass.  Requires s_0 < a < s_m.
template <bool MIR, typename T>
BTD int sweep_raw(const View<T> &F, const T &a, const Arr<T> &o)
{
    Src<MIR, T> f{F, F.m};
    const int m = F.m;
    int n = 0;
    T SMc = mk<T>(0.0), xq = mk<T>(0.0), vq = mk<T>(0.0);
    int Qc = -1;
    double xr = 0.0;  // value of x_{j+1}
    for (int j = m - 1; j >= 0; j--) {
        const T xj = f.X(j), vj = f.V(j);
        const T hj = vj - a * xj;
        T rs;
        if (j == m - 1) {
            rs = f.S(m);
        } else {
            const T sp = f.S(j + 1);
            int kind = 0;  // 0 FLAT, 1 FOLLOW, 2 SPLIT
            T y = mk<T>(0.0);
            if (Qc == j + 1) {
                if (val(sp) >= val(a)) kind = 1;
            } else if (val(hj) < val(SMc) && val(sp) > val(a)) {
                y = xj + (SMc - hj) / (sp - a);
                if (!(val(y) < xr)) kind = 1;
                else if (val(y) > val(xj)) kind = 2;
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
        if (j == m - 1 || val(hj) <= val(SMc)) { SMc = hj; Qc = j; xq = xj; vq = vj; }
        xr = val(xj);
    }
    return n;
}

template <bool MIR, typename T>
BTD int sweep_a(const View<T> &F, const T &a, const Arr<T> &raw, const Arr<T> &o2)
{
    const int n = sweep_raw<MIR, T>(F, a, raw);
    if (n < 0 || n > o2.cap) return -1;
    constexpr int B = pwl_group<T>();
    int k = 0;
    double sl = val(a);
    for (int i0 = 0; i0 < n; i0 += B) {
        T xs[B], vs[B], ss[B];
#pragma unroll
        for (int u = 0; u < B; u++) {
            const int r = n - 1 - (i0 + u);
            if (i0 + u < n) { xs[u] = raw.X(r); vs[u] = raw.V(r); ss[u] = raw.S(r); }
        }
#pragma unroll
        for (int u = 0; u < B; u++) {
            if (i0 + u < n) {
                const double sr = val(ss[u]);
                if (sl != sr) {
                    o2.X(k) = xs[u]; o2.V(k) = vs[u]; o2.S(k + 1) = ss[u];
                    k++;
                }
                sl = sr;
            }
        }
    }
    o2.S(0) = a;
    if (k == 0) { o2.S(1) = a; k = 1; }
    return k;
}

// B = mirror(RB) with CANON, read straight from the raw sweep of RB (slope
// aR on its left tail): the raw order (decreasing x of RB) is B's increasing
// x; point j of B is (-x_j, v_j) with left slope -s_j and right slope
// -s_{j+1} (-aR for the last).  The slopes are negative (between
// -(1+k)S and -(1-k)S, scaled by powers of rho, with S > 0 and k < 1;
// only an underflow of S could make one zero), so dropping RB's collinear
// points before the mirror or after it keeps the same points and the same
// bits.  -1 when dst cannot hold n points.
template <typename T>
BTD int mirror_canon_raw(const Arr<T> &raw, int n, const T &aR, const Arr<T> &dst)
{
    if (n > dst.cap) return -1;
    constexpr int B = pwl_group<T>();
    const T s0 = -raw.S(0);
    int k = 0;
    double sl = val(s0);
    for (int j0 = 0; j0 < n; j0 += B) {
        T xs[B], vs[B], ss[B];
#pragma unroll
        for (int u = 0; u < B; u++) {
            const int j = j0 + u;
            if (j < n) { xs[u] = -raw.X(j); vs[u] = raw.V(j); ss[u] = j + 1 < n ? -raw.S(j + 1) : -aR; }
        }
#pragma unroll
        for (int u = 0; u < B; u++) {
            if (j0 + u < n) {
                const double sr = val(ss[u]);
                if (sl != sr) {
                    dst.X(k) = xs[u]; dst.V(k) = vs[u]; dst.S(k + 1) = ss[u];
                    k++;
                }
                sl = sr;
            }
        }
    }
    dst.S(0) = s0;
    if (k == 0) { dst.S(1) = s0; k = 1; }
    return k;
}

}  // namespace bt
