// bt_wave.hpp -- one node update of Section 3 computed cooperatively by the
// 64 lanes of a wavefront, for nodes whose functions carry many
// breakpoints.  Every operation is the same as in bt_pwl.hpp (same
// per-element formulas, so the same bits); only the order in which elements
// are produced changes:
//   - MERGE ranks every breakpoint of each input in the other one by
//     bisection to place it in the union, evaluates each union point and its
//     interval independently (slot_interval), then keeps the points whose
//     two slopes differ (CANON) with a prefix sum for their positions;
//   - SCALE, CLIP and CANON work element by element plus a prefix sum;
//   - the buying half of ENV takes its suffix minima from a wave-wide scan.
// Work is written as phases "for every element i" (PAR_FOR) separated by
// WSYNC, with scans as separate primitives, so that a host build can run
// the same code with one lane.
#pragma once

#include "bt_pwl.hpp"

namespace bt {

#ifdef BT_HOST_DEBUG
#define WLANE 0
#define PAR_FOR(i, n) for (int i = 0; i < (n); i++)
#define WSYNC() do { } while (0)
#else
#define WLANE ((int)(threadIdx.x & 63))
#define PAR_FOR(i, n) for (int i = WLANE; i < (n); i += 64)
#define WSYNC() wave_sync()
__device__ __forceinline__ void wave_sync()
{
    // stores of this wave visible to its own later loads from other lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
#endif

// Bump allocator over a wave's slice of the pool (doubles).  All lanes make
// the same calls, so the pointers are uniform.
struct WaveTmp {
    double *base;
    int64_t cap, used;
#ifdef BT_HOST_DEBUG
    int64_t peak = 0;   // high-water mark, for sizing studies on the host
#endif
    BTD double *dbl(int64_t n)
    {
        if (n < 1) n = 1;
        if (used + n > cap) return nullptr;
        double *p = base + used;
        used += (n + 1) & ~(int64_t)1;  // keep 16-byte alignment
#ifdef BT_HOST_DEBUG
        if (used > peak) peak = used;
#endif
        return p;
    }
    BTD int *ints(int64_t n) { return (int *)dbl((n + 1) / 2); }
    template <typename T> BTD T *nums(int64_t n) { return (T *)dbl(n * (int64_t)(sizeof(T) / sizeof(double))); }
    template <typename T> BTD bool arr(int cap_pts, Arr<T> *a)
    {
        T *p = nums<T>(3 * (int64_t)cap_pts + 1);
        if (!p) return false;
        a->x = p; a->v = p + cap_pts; a->s = p + 2 * (int64_t)cap_pts;
        a->st = 1; a->cap = cap_pts;
        return true;
    }
};

// Exclusive prefix sum of c[0..n) in place; returns the total (all lanes).
BTD int wave_scan(int *c, int n)
{
#ifdef BT_HOST_DEBUG
    int acc = 0;
    for (int i = 0; i < n; i++) { int v = c[i]; c[i] = acc; acc += v; }
    return acc;
#else
    const int lane = WLANE;
    int carry = 0;
    for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        const int v = i < n ? c[i] : 0;
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (i < n) c[i] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    WSYNC();
    return carry;
#endif
}

// Smallest of the values, with the smallest index among equal values.
BTD void argmin_pick(double &h, int &q, double h2, int q2)
{
    if (h2 < h || (h2 == h && q2 < q)) { h = h2; q = q2; }
}

// Inclusive suffix minima of the values of h[0..n) with the smallest index
// attaining each: SM[j] = min_{i >= j} h[i], Q[j] = that index.
template <typename T>
BTD void wave_suffix_min(const T *h, double *SM, int *Q, int n)
{
#ifdef BT_HOST_DEBUG
    for (int j = n - 1; j >= 0; j--) {
        if (j == n - 1 || val(h[j]) <= SM[j + 1]) { SM[j] = val(h[j]); Q[j] = j; }
        else { SM[j] = SM[j + 1]; Q[j] = Q[j + 1]; }
    }
#else
    const int lane = WLANE;
    double ch = __builtin_huge_val();
    int cq = 0x7fffffff;
    for (int base = ((n - 1) / 64) * 64; base >= 0; base -= 64) {
        const int i = base + lane;
        double x = i < n ? val(h[i]) : __builtin_huge_val();
        int qi = i < n ? i : 0x7fffffff;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            double y = __shfl_down(x, o, 64);
            int qy = __shfl_down(qi, o, 64);
            if (lane + o < 64) argmin_pick(x, qi, y, qy);
        }
        argmin_pick(x, qi, ch, cq);
        if (i < n) { SM[i] = x; Q[i] = qi; }
        ch = __shfl(x, 0, 64);
        cq = __shfl(qi, 0, 64);
    }
    WSYNC();
#endif
}

// Smallest value of c[0..n) (all lanes).
BTD int wave_min_int(const int *c, int n, int init)
{
#ifdef BT_HOST_DEBUG
    int r = init;
    for (int i = 0; i < n; i++) r = c[i] < r ? c[i] : r;
    return r;
#else
    int r = init;
    PAR_FOR(i, n) r = c[i] < r ? c[i] : r;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int y = __shfl_xor(r, o, 64);
        r = y < r ? y : r;
    }
    return r;
#endif
}

// #{j : f.X(j) < y}
template <typename N>
BTD int lower_count(const View<N> &f, double y)
{
    int lo = 0, hi = f.m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (val(f.X(mid)) < y) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Broadcast-free single-lane write helper: only lane 0 executes `stmt`.
#ifdef BT_HOST_DEBUG
#define LANE0(stmt) do { stmt; } while (0)
#else
#define LANE0(stmt) do { if (WLANE == 0) { stmt; } } while (0)
#endif

// CANON of A (m points) into out; returns the count or -1 on overflow.
template <typename N>
BTD int wave_canon(const Arr<N> &A, int m, const Arr<N> &out, WaveTmp &T)
{
    const int64_t mark = T.used;
    int *c = T.ints(m + 1);
    if (!c) return -1;
    PAR_FOR(j, m) c[j] = val(A.S(j)) != val(A.S(j + 1)) ? 1 : 0;
    WSYNC();
    const int k = wave_scan(c, m);
    int r;
    if (k == 0) {
        if (out.cap < 1) { T.used = mark; return -1; }
        LANE0((out.X(0) = A.X(0), out.V(0) = A.V(0), out.S(0) = A.S(0), out.S(1) = A.S(0)));
        r = 1;
    } else {
        if (k > out.cap) { T.used = mark; return -1; }
        PAR_FOR(j, m) {
            if (val(A.S(j)) != val(A.S(j + 1))) {
                const int p = c[j];
                out.X(p) = A.X(j); out.V(p) = A.V(j); out.S(p + 1) = A.S(j + 1);
            }
        }
        LANE0(out.S(0) = A.S(0));
        r = k;
    }
    WSYNC();
    T.used = mark;
    return r;
}

// MERGE(F, G, op) into out (same result as merge<OP>).
template <int OP, typename N>
BTD int wave_merge(const View<N> &F, const View<N> &G, const Arr<N> &out, WaveTmp &T)
{
    const int mF = F.m, mG = G.m;
    const int64_t mark = T.used;
    int *dup = T.ints(mG + 1);
    int *rF = T.ints(mG);
    if (!dup || !rF) return -1;
    PAR_FOR(b, mG) {
        const double xb = val(G.X(b));
        const int r = lower_count(F, xb);
        rF[b] = r;
        dup[b] = (r < mF && val(F.X(r)) == xb) ? 1 : 0;
    }
    WSYNC();
    const int ndup = wave_scan(dup, mG);
    const int K = mF + mG - ndup;
    N *P = T.nums<N>(K), *fF = T.nums<N>(K), *fG = T.nums<N>(K);
    int *IF = T.ints(K), *IG = T.ints(K);
    N *rs = T.nums<N>(K), *cy = T.nums<N>(K), *cv = T.nums<N>(K), *crs = T.nums<N>(K);
    int *hc = T.ints(K), *cnt = T.ints(K + 1);
    if (!P || !fF || !fG || !IF || !IG || !rs || !cy || !cv || !crs || !hc || !cnt) { T.used = mark; return -1; }
    // dup[] is now the exclusive count of duplicated G points before b;
    // G[b] itself is a duplicate when dup[b+1] > dup[b] (dup[mG] = ndup).
    LANE0(dup[mG] = ndup);
    WSYNC();
    PAR_FOR(a, mF) {
        const double xa = val(F.X(a));
        const int r = lower_count(G, xa);
        const bool eq = r < mG && val(G.X(r)) == xa;
        const int k = a + r - dup[r];
        P[k] = F.X(a); IF[k] = a + 1; IG[k] = r + (eq ? 1 : 0);
    }
    PAR_FOR(b, mG) {
        if (dup[b + 1] == dup[b]) {
            const int k = b - dup[b] + rF[b];
            P[k] = G.X(b); IF[k] = rF[b]; IG[k] = b + 1;
        }
    }
    WSYNC();
    PAR_FOR(k, K) {
        fF[k] = eval_at<N>(F, IF[k], P[k]);
        fG[k] = eval_at<N>(G, IG[k], P[k]);
    }
    WSYNC();
    PAR_FOR(k, K) {
        Slot<N> o;
        if (k < K - 1) o = slot_interval<OP, N>(F, G, P[k], IF[k], IG[k], fF[k], fG[k], P[k + 1],
                                               val(fF[k + 1]) - val(fG[k + 1]));
        else o = slot_right<OP, N>(F, G, P[k], fF[k], fG[k]);
        rs[k] = o.rs; hc[k] = o.hc ? 1 : 0;
        if (o.hc) { cy[k] = o.cy; cv[k] = o.cv; crs[k] = o.crs; }
    }
    const Slot<N> L = slot_left<OP, N>(F, G, P[0], fF[0], fG[0]);
    WSYNC();
    // CANON on the emitted sequence [L crossing], P_0, [c_0], P_1, [c_1], ...
    PAR_FOR(k, K) {
        const double sl = k == 0 ? val(L.hc ? L.crs : L.rs) : val(hc[k - 1] ? crs[k - 1] : rs[k - 1]);
        cnt[k] = (sl != val(rs[k]) ? 1 : 0) + ((hc[k] && val(rs[k]) != val(crs[k])) ? 1 : 0);
    }
    WSYNC();
    const int keepL = (L.hc && val(L.rs) != val(L.crs)) ? 1 : 0;
    const int tot = wave_scan(cnt, K) + keepL;
    int r;
    if (tot > out.cap) {
        r = -1;
    } else if (tot == 0) {
        if (out.cap < 1) r = -1;
        else {
            LANE0((out.X(0) = L.hc ? L.cy : P[0], out.V(0) = L.hc ? L.cv : pick<OP, N>(fF[0], fG[0]),
                   out.S(0) = L.rs, out.S(1) = L.rs));
            r = 1;
        }
    } else {
        LANE0(out.S(0) = L.rs);
        if (keepL) LANE0((out.X(0) = L.cy, out.V(0) = L.cv, out.S(1) = L.crs));
        PAR_FOR(k, K) {
            const double sl = k == 0 ? val(L.hc ? L.crs : L.rs) : val(hc[k - 1] ? crs[k - 1] : rs[k - 1]);
            int p = keepL + cnt[k];
            if (sl != val(rs[k])) {
                out.X(p) = P[k]; out.V(p) = pick<OP, N>(fF[k], fG[k]); out.S(p + 1) = rs[k];
                p++;
            }
            if (hc[k] && val(rs[k]) != val(crs[k])) { out.X(p) = cy[k]; out.V(p) = cv[k]; out.S(p + 1) = crs[k]; }
        }
        r = tot;
    }
    WSYNC();
    T.used = mark;
    return r;
}

// SCALE by rho from A into B (then CANON into out).
template <typename N>
BTD int wave_scale(const Arr<N> &A, int m, const N &rho, const Arr<N> &out, WaveTmp &T)
{
    const int64_t mark = T.used;
    Arr<N> B;
    if (!T.arr<N>(m, &B)) return -1;
    PAR_FOR(j, m) { B.X(j) = A.X(j); B.V(j) = A.V(j) * rho; }
    PAR_FOR(j, m + 1) B.S(j) = A.S(j) * rho;
    WSYNC();
    const int r = wave_canon(B, m, out, T);
    T.used = mark;
    return r;
}

// CLIP(A, a, b) into out (seller).
template <typename N>
BTD int wave_clip(const Arr<N> &A, int m, const N &a, const N &b, const Arr<N> &out, WaveTmp &T)
{
    const int64_t mark = T.used;
    if (val(a) == val(b)) {
        int *c = T.ints(m + 1);
        if (!c || out.cap < 1) { T.used = mark; return -1; }
        PAR_FOR(j, m + 1) c[j] = val(A.S(j)) >= val(a) ? j : m + 1;
        WSYNC();
        const int i0 = wave_min_int(c, m + 1, m + 1);
        int q = i0 - 1;
        if (q < 0) q = 0;
        if (q > m - 1) q = m - 1;
        LANE0((out.X(0) = A.X(q), out.V(0) = A.V(q), out.S(0) = a, out.S(1) = a));
        WSYNC();
        T.used = mark;
        return 1;
    }
    PAR_FOR(j, m + 1) {
        const double s = val(A.S(j));
        if (s < val(a)) A.S(j) = a;
        else if (s > val(b)) A.S(j) = b;
    }
    WSYNC();
    return wave_canon(A, m, out, T);
}

// The buying half of ENV (same definition as sweep_a) into out.
template <bool MIR, typename N>
BTD int wave_sweep_a(const View<N> &F, const N &a, const Arr<N> &out, WaveTmp &T)
{
    Src<MIR, N> f{F, F.m};
    const int m = F.m;
    const int64_t mark = T.used;
    N *h = T.nums<N>(m), *rs = T.nums<N>(m), *y = T.nums<N>(m), *yv = T.nums<N>(m);
    double *SM = T.dbl(m);
    int *Q = T.ints(m), *sp = T.ints(m), *cnt = T.ints(m + 1);
    if (!h || !SM || !rs || !y || !yv || !Q || !sp || !cnt) { T.used = mark; return -1; }
    PAR_FOR(j, m) h[j] = f.V(j) - a * f.X(j);
    WSYNC();
    wave_suffix_min(h, SM, Q, m);
    PAR_FOR(j, m) {
        int kind = 0;
        if (j == m - 1) {
            rs[j] = f.S(m);
        } else {
            const N spj = f.S(j + 1);
            const int Qj = Q[j + 1];
            const N hj = h[j];
            if (Qj == j + 1) {
                if (val(spj) >= val(a)) kind = 1;
            } else if (val(hj) < SM[j + 1] && val(spj) > val(a)) {
                const N xj = f.X(j);
                const N yy = xj + (h[Qj] - hj) / (spj - a);
                if (!(val(yy) < val(f.X(j + 1)))) kind = 1;
                else if (val(yy) > val(xj)) {
                    kind = 2;
                    y[j] = yy;
                    yv[j] = f.V(Qj) + a * (yy - f.X(Qj));
                }
            }
            rs[j] = kind != 0 ? spj : a;
        }
        sp[j] = kind == 2 ? 1 : 0;
    }
    WSYNC();
    // CANON of x_0, [y_0], x_1, ... with left tail a; y_j leaves with a
    const double av = val(a);
    PAR_FOR(j, m) {
        const double sl = j == 0 ? av : (sp[j - 1] ? av : val(rs[j - 1]));
        cnt[j] = (sl != val(rs[j]) ? 1 : 0) + ((sp[j] && val(rs[j]) != av) ? 1 : 0);
    }
    WSYNC();
    const int tot = wave_scan(cnt, m);
    int r;
    if (tot > out.cap || out.cap < 1) {
        r = -1;
    } else if (tot == 0) {
        LANE0((out.X(0) = f.X(0), out.V(0) = f.V(0), out.S(0) = a, out.S(1) = a));
        r = 1;
    } else {
        LANE0(out.S(0) = a);
        PAR_FOR(j, m) {
            const double sl = j == 0 ? av : (sp[j - 1] ? av : val(rs[j - 1]));
            int p = cnt[j];
            if (sl != val(rs[j])) { out.X(p) = f.X(j); out.V(p) = f.V(j); out.S(p + 1) = rs[j]; p++; }
            if (sp[j] && val(rs[j]) != av) { out.X(p) = y[j]; out.V(p) = yv[j]; out.S(p + 1) = a; }
        }
        r = tot;
    }
    WSYNC();
    T.used = mark;
    return r;
}

// ENV(F, a, b) into out (buyer).
template <typename N>
BTD int wave_env(const Arr<N> &Fa, int m, const N &a, const N &b, const Arr<N> &out, WaveTmp &T)
{
    const int64_t mark = T.used;
    const View<N> F = Fa.view(m);
    if (val(a) == val(b)) {
        N *h = T.nums<N>(m);
        double *SM = T.dbl(m);
        int *Q = T.ints(m);
        if (!h || !SM || !Q || out.cap < 1) { T.used = mark; return -1; }
        PAR_FOR(j, m) h[j] = F.V(j) - a * F.X(j);
        WSYNC();
        wave_suffix_min(h, SM, Q, m);
        const int js = Q[0];
        LANE0((out.X(0) = F.X(js), out.V(0) = F.V(js), out.S(0) = a, out.S(1) = a));
        WSYNC();
        T.used = mark;
        return 1;
    }
    Arr<N> A, RB, B;
    if (!T.arr<N>(2 * m, &A) || !T.arr<N>(2 * m, &RB) || !T.arr<N>(2 * m, &B)) { T.used = mark; return -1; }
    const int ma = wave_sweep_a<false, N>(F, a, A, T);
    const int mrb = ma < 0 ? -1 : wave_sweep_a<true, N>(F, -b, RB, T);
    if (ma < 0 || mrb < 0) { T.used = mark; return -1; }
    // B = mirror(RB), then CANON
    Arr<N> Bm;
    if (!T.arr<N>(mrb, &Bm)) { T.used = mark; return -1; }
    PAR_FOR(j, mrb) { Bm.X(j) = -RB.X(mrb - 1 - j); Bm.V(j) = RB.V(mrb - 1 - j); }
    PAR_FOR(j, mrb + 1) Bm.S(j) = -RB.S(mrb - j);
    WSYNC();
    const int mb = wave_canon(Bm, mrb, B, T);
    const int mv = mb < 0 ? -1 : wave_merge<OPMIN, N>(A.view(ma), B.view(mb), out, T);
    T.used = mark;
    return mv;
}

// One node update by a whole wave (see node_update).  The result is left in
// *zout inside T's slice (valid until T is reset).
template <int SIDE, typename N>
BTD int wave_node_update(const View<N> &Zu, const View<N> &Zd, const N &S, const N &kt, const N &rho,
                         const N &xi, const N &zeta, bool exercise, WaveTmp &T, Arr<N> *zout)
{
    const N one = mk<N>(1.0);
    const N a = -((one + kt) * S);
    const N b = -((one - kt) * S);
    const int M = Zu.m + Zd.m;
    Arr<N> W, W2, V;
    if (!T.arr<N>(2 * M + 1, &W)) return -1;
    int mw = wave_merge<OPMAX, N>(Zu, Zd, W, T);
    if (mw < 0 || !T.arr<N>(mw, &W2)) return -1;
    mw = wave_scale(W, mw, rho, W2, T);
    if (mw < 0) return -1;
    int mv;
    if (SIDE == 0) {
        if (!T.arr<N>(mw, &V)) return -1;
        mv = wave_clip(W2, mw, a, b, V, T);
    } else {
        // the output of ENV is bounded by 8 mw + 1 points but is about mw in
        // practice: try a buffer of 2 mw + 8 first and fall back to the bound
        const int64_t markv = T.used;
        if (!T.arr<N>(2 * mw + 8, &V)) return -1;
        mv = wave_env(W2, mw, a, b, V, T);
        if (mv < 0) {
            T.used = markv;
            if (!T.arr<N>(8 * mw + 1, &V)) return -1;
            mv = wave_env(W2, mw, a, b, V, T);
        }
    }
    if (mv < 0) return -1;
    if (!exercise) { *zout = V; return mv; }
    Arr<N> U, Z;
    if (!T.arr<N>(1, &U) || !T.arr<N>(2 * mv + 3, &Z)) return -1;
    LANE0((U.X(0) = SIDE == 0 ? zeta : -zeta, U.V(0) = SIDE == 0 ? xi : -xi, U.S(0) = a, U.S(1) = b));
    WSYNC();
    const int mz = wave_merge<SIDE == 0 ? OPMAX : OPMIN, N>(U.view(1), V.view(mv), Z, T);
    *zout = Z;
    return mz;
}

}  // namespace bt
