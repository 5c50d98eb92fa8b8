// bt_wave.hpp -- one node update of Section 3 computed cooperatively by the
// 64 lanes of a wavefront, for nodes whose functions carry many
// breakpoints.  Every operation gives the same result as in bt_pwl.hpp (the
// same per-element formulas, so the same bits); only the order in which
// elements are produced changes.
//
// The work goes in tiles of 64 E consecutive elements (E per lane: for
// CANON, CLIP and the envelope sweeps 4 for double and 1 for the dual
// numbers of the Greeks (TileE); for MERGE 8 and 2 merged positions
// (WaveLds)), so that a tile's loads are issued together and its latency is
// paid once per tile:
//   - CANON (and SCALE, CLIP, the mirror image taken by ENV, applied on the
//     fly as accessors of its input) loads a tile into registers, counts the
//     points each lane keeps, takes an exclusive scan over the lanes and
//     writes at the running offset;
//   - MERGE stages, per tile of the merged order of both breakpoint lists
//     (F first on equal abscissae), the windows of F and G the tile touches
//     in LDS with coalesced loads; each lane then finds its diagonal by
//     merge-path bisection inside the windows and walks it once (with a
//     lookbehind of two merged positions and a lookahead of one union
//     point), staging the points it emits in LDS, from where they are
//     copied to their place after a scan of the counts;
//   - the buying half of ENV runs its tiles from right to left with the
//     running suffix minimum of h carried between tiles, and writes its
//     points from the right end of the output buffer (their number is only
//     known at the end); the caller reads the result at the returned offset.
// Lane-parallel code is written as LANES(l) { ... } blocks over per-lane
// values LV<T>, with the cross-lane steps (scans, broadcasts) between the
// blocks: on the GPU a block runs once per lane, in a host build
// (BT_HOST_DEBUG) it runs for every emulated lane in turn, so the host
// build checks the lane logic for any number of lanes.
#pragma once

#include "bt_pwl.hpp"

namespace bt {

#ifdef BT_HOST_DEBUG
inline int bt_host_lanes = 64;   // lanes emulated by the host build (<= 256)
inline long long bt_host_env_sched[2];   // scheduled envelope merges, and fallbacks to the walk
#define NLANES (bt_host_lanes)
#define LANES(l) for (int l = 0; l < bt_host_lanes; l++)
#define WSYNC() do { } while (0)
#define LANE0(stmt) do { stmt; } while (0)
template <typename T>
struct LV {
    T *a;
    LV() : a(new T[256]) {}
    ~LV() { delete[] a; }
    LV(const LV &) = delete;
    LV &operator=(const LV &) = delete;
    T &operator()(int l) { return a[l]; }
    const T &operator()(int l) const { return a[l]; }
};
#else
#define WLANE ((int)(threadIdx.x & 63))
#define NLANES 64
#define LANES(l) for (int l = WLANE, l##_once = 1; l##_once; l##_once = 0)
#define WSYNC() wave_sync()
#define LANE0(stmt) do { if (WLANE == 0) { stmt; } } while (0)
__device__ __forceinline__ void wave_sync()
{
    // stores of this wave visible to its own later loads from other lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
template <typename T>
struct LV {
    T a;
    __device__ __forceinline__ T &operator()(int) { return a; }
    __device__ __forceinline__ const T &operator()(int) const { return a; }
};
// Cross-lane moves by DPP (row shifts and broadcasts, whole-wave shifts) and
// v_readlane: no LDS round trip.  CTRL: 0x101-0x10f row_shl, 0x111-0x11f
// row_shr, 0x130 wave_shl:1, 0x138 wave_shr:1, 0x142 row_bcast:15, 0x143
// row_bcast:31.  Lanes without a source keep `old`.
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ int dpp_i(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ double dpp_d(double old, double src)
{
    const long long o = __double_as_longlong(old), x = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, CTRL, RM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, RM, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// value of lane src (src the same in every lane)
__device__ __forceinline__ int shfl_num(int x, int src) { return __builtin_amdgcn_readlane(x, src); }
__device__ __forceinline__ double shfl_num(double x, int src)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ D4 shfl_num(const D4 &x, int src)
{
    D4 r;
    r.v = shfl_num(x.v, src);
    for (int i = 0; i < 4; i++) r.d[i] = shfl_num(x.d[i], src);
    return r;
}
#endif

// Elements per lane in a tile of CANON and the sweeps.
template <typename N>
struct TileE {
    static constexpr int E = sizeof(N) == sizeof(double) ? 4 : 1;
};

// MERGE: merged positions per lane (E), and the numbers of LDS one wave's
// MERGE takes: the abscissas of two windows of W = 64 E + 9 points each
// (binary64, the walk compares nothing else) and the staging of the points
// the lanes emit (x, v, s of 2 E slots per lane).
template <typename N>
struct WaveLds {
    static constexpr int E = sizeof(N) == sizeof(double) ? 8 : 2;
    static constexpr int W = 64 * E + 9;
    static constexpr int STAGE = 2 * E * 64;
    static constexpr int WIN = (2 * W * (int)sizeof(double) + (int)sizeof(N) - 1) / (int)sizeof(N);
    static constexpr int NUMS = WIN + 3 * STAGE;
};

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

// ---------------------------------------------------------------------------
// Cross-lane steps.
// ---------------------------------------------------------------------------

// Exclusive prefix sums over the lanes in place; returns the total.
BTD int lv_exscan(LV<int> &v)
{
#ifdef BT_HOST_DEBUG
    int acc = 0;
    for (int l = 0; l < bt_host_lanes; l++) { const int t = v(l); v(l) = acc; acc += t; }
    return acc;
#else
    const int x0 = v.a;
    int x = x0;
    x += dpp_i<0x111>(0, x);
    x += dpp_i<0x112>(0, x);
    x += dpp_i<0x114>(0, x);
    x += dpp_i<0x118>(0, x);
    x += dpp_i<0x142, 0xa>(0, x);
    x += dpp_i<0x143, 0xc>(0, x);
    v.a = x - x0;
    return __builtin_amdgcn_readlane(x, 63);
#endif
}

// Exclusive suffix sums (over the lanes to the right) in place; returns the
// total.
BTD int lv_rexscan(LV<int> &v)
{
#ifdef BT_HOST_DEBUG
    int acc = 0;
    for (int l = bt_host_lanes - 1; l >= 0; l--) { const int t = v(l); v(l) = acc; acc += t; }
    return acc;
#else
    // inclusive prefix sums; the lanes to the right hold total - prefix
    int x = v.a;
    x += dpp_i<0x111>(0, x);
    x += dpp_i<0x112>(0, x);
    x += dpp_i<0x114>(0, x);
    x += dpp_i<0x118>(0, x);
    x += dpp_i<0x142, 0xa>(0, x);
    x += dpp_i<0x143, 0xc>(0, x);
    const int tot = __builtin_amdgcn_readlane(x, 63);
    v.a = tot - x;
    return tot;
#endif
}

// Smallest value, with the smallest index among equal values.
BTD void argmin_pick(double &h, int &q, double h2, int q2)
{
    if (h2 < h || (h2 == h && q2 < q)) { h = h2; q = q2; }
}

// Per-lane (value, index) -> the minimum over the lanes to the right
// ((+inf, INT_MAX) for the last lane), in place.
BTD void lv_rexmin(LV<double> &h, LV<int> &q)
{
#ifdef BT_HOST_DEBUG
    double ch = __builtin_huge_val();
    int cq = 0x7fffffff;
    for (int l = bt_host_lanes - 1; l >= 0; l--) {
        const double th = h(l);
        const int tq = q(l);
        h(l) = ch;
        q(l) = cq;
        argmin_pick(ch, cq, th, tq);
    }
#else
    // (the pick is a lexicographic minimum, so the order of combination
    // does not matter) suffix minima within each row of 16 lanes ...
    const double INF = __builtin_huge_val();
    const int QMAX = 0x7fffffff;
    double x = h.a;
    int qi = q.a;
    argmin_pick(x, qi, dpp_d<0x101>(INF, x), dpp_i<0x101>(QMAX, qi));
    argmin_pick(x, qi, dpp_d<0x102>(INF, x), dpp_i<0x102>(QMAX, qi));
    argmin_pick(x, qi, dpp_d<0x104>(INF, x), dpp_i<0x104>(QMAX, qi));
    argmin_pick(x, qi, dpp_d<0x108>(INF, x), dpp_i<0x108>(QMAX, qi));
    // ... then the rows to the right, whose first lanes hold their minima
    const double r1 = shfl_num(x, 16), r2 = shfl_num(x, 32), r3 = shfl_num(x, 48);
    const int q1 = shfl_num(qi, 16), q2 = shfl_num(qi, 32), q3 = shfl_num(qi, 48);
    const int row = WLANE >> 4;
    if (row < 3) argmin_pick(x, qi, r3, q3);
    if (row < 2) argmin_pick(x, qi, r2, q2);
    if (row < 1) argmin_pick(x, qi, r1, q1);
    // exclusive: the next lane's inclusive minimum
    h.a = dpp_d<0x130>(INF, x);
    q.a = dpp_i<0x130>(QMAX, qi);
#endif
}

// Per-lane values -> for every lane the value of the lane before it
// (`fill` for lane 0), in place.
BTD void lv_up1(LV<double> &v, double fill)
{
#ifdef BT_HOST_DEBUG
    for (int l = bt_host_lanes - 1; l > 0; l--) v(l) = v(l - 1);
    v(0) = fill;
#else
    v.a = dpp_d<0x138>(fill, v.a);
#endif
}

// The value get(src) of lane src, for every lane.
template <typename T, class G>
BTD T from_lane(int src, G get)
{
#ifdef BT_HOST_DEBUG
    return get(src);
#else
    return shfl_num(get(WLANE), src);
#endif
}

// Overall minimum of per-lane integers, or first index of the overall
// minimum of per-lane (value, index) pairs.
BTD int lv_min_int(LV<int> &v)
{
#ifdef BT_HOST_DEBUG
    int r = 0x7fffffff;
    for (int l = 0; l < bt_host_lanes; l++) r = v(l) < r ? v(l) : r;
    return r;
#else
    int r = v.a;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(r, o, 64);
        r = y < r ? y : r;
    }
    return r;
#endif
}

BTD int lv_argmin(LV<double> &h, LV<int> &q)
{
#ifdef BT_HOST_DEBUG
    double ch = __builtin_huge_val();
    int cq = 0x7fffffff;
    for (int l = 0; l < bt_host_lanes; l++) argmin_pick(ch, cq, h(l), q(l));
    return cq;
#else
    double x = h.a;
    int qi = q.a;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(x, o, 64);
        const int qy = __shfl_xor(qi, o, 64);
        argmin_pick(x, qi, y, qy);
    }
    return qi;
#endif
}

// ---------------------------------------------------------------------------
// CANON over an accessor (X(j), V(j), S(j)).
// ---------------------------------------------------------------------------

// A with values and slopes multiplied by rho (SCALE).
template <typename N>
struct ScaleSrc {
    View<N> A;
    N rho;
    BTD N X(int j) const { return A.X(j); }
    BTD N V(int j) const { return A.V(j) * rho; }
    BTD N S(int j) const { return A.S(j) * rho; }
};

// A with its slopes clamped into [a, b] (CLIP, a < b).
template <typename N>
struct ClampSrc {
    View<N> A;
    N a, b;
    BTD N X(int j) const { return A.X(j); }
    BTD N V(int j) const { return A.V(j); }
    BTD N S(int j) const
    {
        const N s = A.S(j);
        const double sv = val(s);
        return sv < val(a) ? a : (sv > val(b) ? b : s);
    }
};

// The mirror image y -> -y of a stored function with m points.
template <typename N>
struct MirSrc {
    View<N> A;
    int m;
    BTD N X(int j) const { return -A.X(m - 1 - j); }
    BTD N V(int j) const { return A.V(m - 1 - j); }
    BTD N S(int j) const { return -A.S(m - j); }
};

// CANON of src (m points) into out; returns the count or -1 on overflow.
template <typename N, typename SRC>
BTD int wave_canon(const SRC &src, int m, const Arr<N> &out)
{
    constexpr int E = TileE<N>::E;
    struct Ld {
        N x[E], v[E], s1[E];
        double s0[E];
    };
    const int tm = NLANES * E;
    if (out.cap < 1) return -1;
    int carry = 0;
    for (int t0 = 0; t0 < m; t0 += tm) {
        LV<Ld> ld;
        LV<int> c;
        LANES(l) {
            Ld &q = ld(l);
            const int j0 = t0 + l * E;
#pragma unroll
            for (int u = 0; u < E; u++) {
                const int j = j0 + u;
                if (j < m) {
                    q.x[u] = src.X(j);
                    q.v[u] = src.V(j);
                    q.s1[u] = src.S(j + 1);
                    q.s0[u] = val(src.S(j));
                }
            }
            int cc = 0;
#pragma unroll
            for (int u = 0; u < E; u++)
                if (j0 + u < m && q.s0[u] != val(q.s1[u])) cc++;
            c(l) = cc;
        }
        const int tot = lv_exscan(c);
        if (carry + tot > out.cap) return -1;
        LANES(l) {
            const Ld &q = ld(l);
            const int j0 = t0 + l * E;
            int p = carry + c(l);
#pragma unroll
            for (int u = 0; u < E; u++) {
                if (j0 + u < m && q.s0[u] != val(q.s1[u])) {
                    out.X(p) = q.x[u]; out.V(p) = q.v[u]; out.S(p + 1) = q.s1[u];
                    p++;
                }
            }
        }
        carry += tot;
    }
    if (carry == 0) {
        LANE0((out.X(0) = src.X(0), out.V(0) = src.V(0), out.S(0) = src.S(0), out.S(1) = src.S(0)));
        WSYNC();
        return 1;
    }
    LANE0(out.S(0) = src.S(0));
    WSYNC();
    return carry;
}

// ---------------------------------------------------------------------------
// MERGE(F, G, op) (same result as merge<OP>).
// ---------------------------------------------------------------------------

// The abscissas of a function's points [base, base + W) staged in LDS;
// indices are those of the whole function.
struct XWin {
    double *x;
    int base, m;
    BTD double X(int j) const { return x[j - base]; }
};

// Number of F elements among the first d of the merged order, searched in
// [lo, hi] (a bracket known to hold it).
template <typename FF, typename GG>
BTD int merge_path_in(const FF &F, const GG &G, int d, int lo, int hi)
{
    // The predicate F.X(a) <= G.X(d - a - 1) holds for a below the answer
    // and fails from it on, so the number of probes that hold places it.
    // Quaternary steps: three probes whose loads issue together.
    while (hi - lo > 3) {
        const int w = (hi - lo) >> 2;
        const int m1 = lo + w, m2 = lo + 2 * w, m3 = lo + 3 * w;
        const int c = (val(F.X(m1)) <= val(G.X(d - m1 - 1)) ? 1 : 0) + (val(F.X(m2)) <= val(G.X(d - m2 - 1)) ? 1 : 0) +
                      (val(F.X(m3)) <= val(G.X(d - m3 - 1)) ? 1 : 0);
        const int nlo = c == 0 ? lo : (c == 1 ? m1 + 1 : (c == 2 ? m2 + 1 : m3 + 1));
        hi = c == 0 ? m1 : (c == 1 ? m2 : (c == 2 ? m3 : hi));
        lo = nlo;
    }
    // at most three candidates left: all probed at once
    if (lo < hi) {
        const int a1 = lo + 1 < hi ? lo + 1 : lo, a2 = lo + 2 < hi ? lo + 2 : lo;
        const int c = (val(F.X(lo)) <= val(G.X(d - lo - 1)) ? 1 : 0) +
                      ((val(F.X(a1)) <= val(G.X(d - a1 - 1)) && lo + 1 < hi) ? 1 : 0) +
                      ((val(F.X(a2)) <= val(G.X(d - a2 - 1)) && lo + 2 < hi) ? 1 : 0);
        lo += c;
    }
    return lo;
}

// Bracket of the merge-path coordinate at d from the one at dt (at): it
// moves by at most one per merged position.
BTD void mp_bracket(int d, int dt, int at, int mF, int mG, int &lo, int &hi)
{
    lo = d - mG > 0 ? d - mG : 0;
    hi = d < mF ? d : mF;
    if (d >= dt) {
        lo = lo > at ? lo : at;
        hi = hi < at + (d - dt) ? hi : at + (d - dt);
    } else {
        lo = lo > at - (dt - d) ? lo : at - (dt - d);
        hi = hi < at ? hi : at;
    }
}

// The first union point a lane owns, held back until the slope arriving
// from the lane before is known.
template <typename N>
struct LaneFirst {
    N x, v, rs, cy, cv, crs;
    bool hc, have;
    double rf, rg, fl, cfl;   // records of the point and of the crossing (VO)
};

// The decisions of a lane's walk over its K = E + 2 merged positions
// [d0, d1 + 2): the point counts after each position and whether it starts
// a union point and from which list (0 none: past the end or a duplicate;
// 1 F; 2 G); aend = the number of F points among positions < d1.
template <int E>
struct LaneWalk {
    int iF[E + 2], iG[E + 2], src[E + 2];
    int d0, d1, pe, aend;
};

// First step of merge_lane without its lookbehind: walk the merged order
// (one load per step: the next abscissa of the list that advanced, kept two
// steps ahead).
template <int E, typename FF, typename GG>
BTD void merge_walk(const FF &F, const GG &G, int d0, int d1, int dt, int at, LaneWalk<E> &w)
{
    constexpr int K = E + 2;
    w.d0 = d0;
    w.d1 = d1;
    w.aend = at;
#pragma unroll
    for (int k = 0; k < K; k++) { w.src[k] = 0; w.iF[k] = 0; w.iG[k] = 0; }
    const int mF = F.m, mG = G.m, Lt = mF + mG;
    w.pe = d1 + 2 < Lt ? d1 + 2 : Lt;
    if (d0 >= d1) return;
    int lo, hi;
    mp_bracket(d0, dt, at, mF, mG, lo, hi);
    int a = merge_path_in(F, G, d0, lo, hi);
    int b = d0 - a;
    // abscissas past a list's end read as 0 and are never compared; every
    // load is clamped into the list (and the window), so none needs a branch
    const auto fx = [&](int j) { return val(F.X(j < mF ? j : mF - 1)); };
    const auto gx = [&](int j) { return val(G.X(j < mG ? j : mG - 1)); };
    double xa = fx(a), xb = gx(b), xa1 = fx(a + 1), xb1 = gx(b + 1);
    double xpf = a > 0 ? fx(a - 1) : -__builtin_huge_val();
    int aend = a;
#pragma unroll
    for (int k = 0; k < K; k++) {
        // past the end: the last counts, so that the settle step's loads
        // stay in range
        w.iF[k] = a;
        w.iG[k] = b;
        if (d0 + k < w.pe) {
            const bool tf = a < mF && (b >= mG || xa <= xb);
            const double xn = tf ? fx(a + 2) : gx(b + 2);   // the list that advances, two ahead
            w.iF[k] = tf ? a + 1 : a;
            w.iG[k] = tf ? b + ((b < mG && xb == xa) ? 1 : 0) : b + 1;
            w.src[k] = tf ? 1 : (xpf == xb ? 0 : 2);
            xpf = tf ? xa : xpf;
            a += tf ? 1 : 0;
            b += tf ? 0 : 1;
            xa = tf ? xa1 : xa;
            xa1 = tf ? xn : xa1;
            xb = tf ? xb : xb1;
            xb1 = tf ? xb1 : xn;
            if (d0 + k == d1 - 1) aend = a;
        }
    }
    w.aend = aend;
}


// Second step: evaluate every recorded union point (the pieces of F and G
// loaded two elements ahead of their use) and settle intervals and CANON
// decisions in order.  Same result as merge_lane for the union points at
// positions [d0, d1): the first one is returned in *first (its CANON
// decision needs the slope arriving from the lane before), the points after
// it go to the staging slots; *psl_out is the slope arriving at the first
// union point after the lane's.  Returns the number of staged points.
// With SC the emitted values and slopes are multiplied by rho and the CANON
// decisions compare the products (MERGE followed by SCALE: a point whose
// scaled slopes are equal is the one SCALE's CANON would drop).
//
// With VO (decisions only) the staged slots and the records of *first hold,
// instead of a point, how to rebuild it from the pieces: the point counts of
// F and G at its union point P (the pieces it evaluates) and flags: 1 = the
// crossing after P (else P itself), 2 = P is F's point (else G's), 4 = the
// value is F's (else G's), 8 = the slope leaving is F's (else G's).
template <int OP, int E, bool SC, typename N, typename FF, typename GG, bool VO = false>
BTD int merge_settle(const FF &F, const GG &G, const LaneWalk<E> &w, N *sx, N *sv, N *ss, int stride,
                     LaneFirst<N> *first, double *psl_out, const N &rho)
{
    const auto scl = [&](const N &x) -> N {
        if constexpr (SC) return x * rho;
        else return x;
    };
    constexpr int K = E + 2;
    first->have = false;
    *psl_out = 0.0;
    const int d0 = w.d0, d1 = w.d1, pe = w.pe, Lt = F.m + G.m;
    if (d0 >= d1) return 0;
    constexpr int PD = 2;
    Seg<N> gFk[K], gGk[K];
    // (every position's counts are in range, so the loads need no branch)
#pragma unroll
    for (int k = 0; k < PD && k < K; k++) {
        gFk[k] = seg_at<N>(F, w.iF[k]);
        gGk[k] = seg_at<N>(G, w.iG[k]);
    }
    N cP = mk<N>(0.0), cfF = mk<N>(0.0), cfG = mk<N>(0.0);
    Seg<N> cgF{}, cgG{};
    int cpos = -1, ciF = 0, ciG = 0;
    bool have = false, cpF = false;
    double psl = 0.0;
    int cnt = 0;
    // emits the union point cP (with slot o) and its crossing, or their records
    const auto emit = [&](const Slot<N> &o) {
        const N rs = scl(o.rs), crs = o.hc ? scl(o.crs) : rs, cv = o.hc ? scl(o.cv) : rs;
        const bool vF = pick_first<OP, N>(cfF, cfG);
        double pfl = 0.0, cfl = 0.0;
        if constexpr (VO) {
            pfl = (cpF ? 2 : 0) + (vF ? 4 : 0) + (o.rsF ? 8 : 0);
            cfl = 1 + (cpF ? 2 : 0) + (o.cvF ? 4 : 0) + (o.crsF ? 8 : 0);
        }
        if (!first->have) {
            *first = LaneFirst<N>{cP, scl(vF ? cfF : cfG), rs, o.cy, cv, crs, o.hc, true,
                                  VO ? (double)ciF : 0.0, VO ? (double)ciG : 0.0, pfl, cfl};
        } else {
            if (psl != val(rs)) {
                if constexpr (VO) { sx[cnt * stride] = ciF; sv[cnt * stride] = ciG; ss[cnt * stride] = pfl; }
                else { sx[cnt * stride] = cP; sv[cnt * stride] = scl(vF ? cfF : cfG); ss[cnt * stride] = rs; }
                cnt++;
            }
            if (o.hc && val(rs) != val(crs)) {
                if constexpr (VO) { sx[cnt * stride] = ciF; sv[cnt * stride] = ciG; ss[cnt * stride] = cfl; }
                else { sx[cnt * stride] = o.cy; sv[cnt * stride] = cv; ss[cnt * stride] = crs; }
                cnt++;
            }
        }
        psl = val(o.hc ? crs : rs);
    };
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (k + PD < K) {
            gFk[k + PD] = seg_at<N>(F, w.iF[k + PD]);
            gGk[k + PD] = seg_at<N>(G, w.iG[k + PD]);
        }
        if (w.src[k] != 0) {
            const N x = w.src[k] == 1 ? gFk[k].x : gGk[k].x;
            const N fF = seg_eval<N>(gFk[k], x), fG = seg_eval<N>(gGk[k], x);
            if (have && cpos < d1) emit(slot_interval_seg<OP, N>(cgF, cgG, cP, cfF, cfG, x, val(fF) - val(fG)));
            cP = x; cfF = fF; cfG = fG; cgF = gFk[k]; cgG = gGk[k]; cpos = d0 + k;
            ciF = w.iF[k]; ciG = w.iG[k]; cpF = w.src[k] == 1;
            have = true;
        }
    }
    // the last union point of the whole merge has the right tail after it
    if (have && pe == Lt && cpos < d1) emit(slot_right<OP, N>(F, G, cP, cfF, cfG));
    *psl_out = psl;
    return cnt;
}

// The abscissas of both windows of a tile held in registers (loads issued
// early, e.g. while the tile before settles; stores to LDS later).
template <typename N>
struct WinRegs {
#ifdef BT_HOST_DEBUG
    static constexpr int KW = WaveLds<N>::W;   // any number of emulated lanes
#else
    static constexpr int KW = (WaveLds<N>::W + 63) / 64;
#endif
    double fx[KW], gx[KW];
    int fb, gb, fm, gm;
};

template <typename N, typename FF, typename GG>
BTD void win_load(const FF &F, const GG &G, int fb, int gb, WinRegs<N> &r, int l)
{
    constexpr int W = WaveLds<N>::W;
    r.fb = fb; r.gb = gb; r.fm = F.m; r.gm = G.m;
#pragma unroll
    for (int k = 0; k < WinRegs<N>::KW; k++) {
        const int i = l + NLANES * k, jf = fb + i, jg = gb + i;
        if (i < W && jf < F.m) r.fx[k] = val(F.X(jf));
        if (i < W && jg < G.m) r.gx[k] = val(G.X(jg));
    }
}

template <typename N>
BTD void win_store(double *buf, const WinRegs<N> &r, XWin *wf, XWin *wg, int l)
{
    constexpr int W = WaveLds<N>::W;
    *wf = XWin{buf, r.fb, r.fm};
    *wg = XWin{buf + W, r.gb, r.gm};
#pragma unroll
    for (int k = 0; k < WinRegs<N>::KW; k++) {
        const int i = l + NLANES * k, jf = r.fb + i, jg = r.gb + i;
        if (i < W && jf < r.fm) buf[i] = r.fx[k];
        if (i < W && jg < r.gm) buf[W + i] = r.gx[k];
    }
}

// Merged positions [r0, r1) of MERGE(F, G, op) (r0 a multiple of the tile;
// at0 = the number of F points among the first r0 merged positions),
// emitted into out from position `carry`; psl, *psl_out and *first_rs as in
// merge_sched_tiles.  Template arguments as in wave_merge.
template <int OP, typename N, bool SC, bool VO, typename FF, typename GG>
BTD int merge_tiles(const FF &F, const GG &G, const Arr<N> &out, N *lds, const N &rho, int r0, int r1, int at0,
                    int carry, double psl, double *psl_out, double *first_rs)
{
    constexpr int E = WaveLds<N>::E;
    const int tm = NLANES * E;
    const int Lt = F.m + G.m;
    // the windows' abscissas, then the staging (slot k of lane l at
    // k * NLANES + l); a tile's windows are loaded into registers while the
    // tile before settles
    double *xw = (double *)lds;
    const int SZ = 2 * E * NLANES;
    N *stg = lds + WaveLds<N>::WIN;
    LV<WinRegs<N>> pre;
    {
        const int bn = r0 - at0;
        LANES(l) { win_load<N>(F, G, at0 >= 3 ? at0 - 3 : 0, bn >= 3 ? bn - 3 : 0, pre(l), l); }
    }
    if (first_rs) *first_rs = __builtin_nan("");
    int at = at0;
    for (int dt = r0; dt < r1; dt += tm) {
        WSYNC();   // the previous tile's reads of the windows and staging are done
        XWin wf, wg;
        LANES(l) { win_store<N>(xw, pre(l), &wf, &wg, l); }
        WSYNC();
        const int dend = dt + tm < r1 ? dt + tm : r1;
        {
            LV<LaneWalk<E>> wk;
            LANES(l) {
                const int d0 = dt + l * E;
                const int d1 = d0 + E < dend ? d0 + E : dend;
                merge_walk<E>(wf, wg, d0, d1, dt, at, wk(l));
            }
            // merge-path coordinate at dend: the walk of the lane ending there
            int at_next = at;
            if (dend < Lt) {
                at_next = from_lane<int>((dend - dt - 1) / E, [&](int l) { return wk(l).aend; });
                const int bn = dend - at_next;
                if (dend < r1) {
                    LANES(l) { win_load<N>(F, G, at_next >= 3 ? at_next - 3 : 0, bn >= 3 ? bn - 3 : 0, pre(l), l); }
                }
            }
            LV<int> c, own;
            LV<double> pso;
            LV<LaneFirst<N>> fst;
            LANES(l) {
                double po;
                own(l) = merge_settle<OP, E, SC, N, FF, GG, VO>(F, G, wk(l), stg + l, stg + SZ + l,
                                                               stg + 2 * SZ + l, NLANES, &fst(l), &po, rho);
                pso(l) = po;
            }
            if (first_rs && dt == r0)
                *first_rs = from_lane<double>(0, [&](int l) { return fst(l).have ? val(fst(l).rs) : __builtin_nan(""); });
            // the slope arriving at each lane's first union point comes from
            // the lane before (the tile before, for lane 0)
            if constexpr (E == 1) {
                // a one-position lane holding a duplicate owns no union point
                // and passes the slope on; the lane before it owns the equal
                // F point (or is the tile before)
                LV<double> sh;
                LANES(l) { sh(l) = pso(l); }
                lv_up1(sh, psl);
                LANES(l) {
                    if (!fst(l).have) pso(l) = sh(l);
                }
            }
            const double pnext = from_lane<double>(NLANES - 1, [&](int l) { return pso(l); });
            lv_up1(pso, psl);
            LANES(l) {
                const LaneFirst<N> &f = fst(l);
                const int cf = f.have ? (pso(l) != val(f.rs) ? 1 : 0) + ((f.hc && val(f.rs) != val(f.crs)) ? 1 : 0) : 0;
                c(l) = cf + own(l);
            }
            const int tot = lv_exscan(c);
            if (carry + tot > out.cap) return -1;
            LANES(l) {
                const LaneFirst<N> &f = fst(l);
                int p = carry + c(l);
                if (f.have) {
                    if constexpr (VO) {
                        if (pso(l) != val(f.rs)) { out.X(p) = f.rf; out.V(p) = f.rg; out.S(p + 1) = f.fl; p++; }
                        if (f.hc && val(f.rs) != val(f.crs)) { out.X(p) = f.rf; out.V(p) = f.rg; out.S(p + 1) = f.cfl; p++; }
                    } else {
                        if (pso(l) != val(f.rs)) { out.X(p) = f.x; out.V(p) = f.v; out.S(p + 1) = f.rs; p++; }
                        if (f.hc && val(f.rs) != val(f.crs)) { out.X(p) = f.cy; out.V(p) = f.cv; out.S(p + 1) = f.crs; p++; }
                    }
                }
                const int n = own(l);
#pragma unroll
                for (int k = 0; k < 2 * E; k++) {
                    if (k < n) {
                        const int q = k * NLANES + l;
                        out.X(p + k) = stg[q]; out.V(p + k) = stg[SZ + q]; out.S(p + k + 1) = stg[2 * SZ + q];
                    }
                }
            }
            carry += tot;
            psl = pnext;
            at = at_next;
        }
    }
    *psl_out = psl;
    return carry;
}

// The left end of MERGE(F, G, op): the first union point P0, the decision
// there (scaled by rho with SC), and the slope arriving at the first tile.
template <int OP, typename N>
struct MergeHead {
    N P0, fF0, fG0;
    Slot<N> L;
    N Lrs, Lcrs;
    int keepL;
    double psl;
};

template <int OP, typename N, bool SC, typename FF, typename GG>
BTD MergeHead<OP, N> merge_head(const FF &F, const GG &G, const N &rho)
{
    MergeHead<OP, N> h;
    int iF0, iG0;
    const double xa = val(F.X(0)), xb = val(G.X(0));
    if (xa < xb) { h.P0 = F.X(0); iF0 = 1; iG0 = 0; }
    else if (xb < xa) { h.P0 = G.X(0); iF0 = 0; iG0 = 1; }
    else { h.P0 = F.X(0); iF0 = 1; iG0 = 1; }
    h.fF0 = eval_at<N>(F, iF0, h.P0);
    h.fG0 = eval_at<N>(G, iG0, h.P0);
    h.L = slot_left<OP, N>(F, G, h.P0, h.fF0, h.fG0);
    if constexpr (SC) {
        h.Lrs = h.L.rs * rho;
        h.Lcrs = h.L.hc ? h.L.crs * rho : h.Lrs;
    } else {
        h.Lrs = h.L.rs;
        h.Lcrs = h.L.hc ? h.L.crs : h.Lrs;
    }
    h.keepL = (h.L.hc && val(h.Lrs) != val(h.Lcrs)) ? 1 : 0;
    h.psl = val(h.L.hc ? h.Lcrs : h.Lrs);   // slope arriving at the next tile's first union point
    return h;
}

// Completes MERGE(F, G, op) whose tiles emitted `carry` points.
template <int OP, typename N, bool SC, bool VO>
BTD int merge_finish(const MergeHead<OP, N> &h, int carry, const Arr<N> &out, const N &rho)
{
    if (carry == 0) {
        if constexpr (SC || VO) return 0;
        LANE0((out.X(0) = h.L.hc ? h.L.cy : h.P0, out.V(0) = h.L.hc ? h.L.cv : pick<OP, N>(h.fF0, h.fG0),
               out.S(0) = h.L.rs, out.S(1) = h.L.rs));
        WSYNC();
        return 1;
    }
    if constexpr (VO) {
        WSYNC();
        return carry;
    }
    N cv = h.L.cv;
    if constexpr (SC) cv = h.L.cv * rho;
    LANE0(out.S(0) = h.Lrs);
    if (h.keepL) LANE0((out.X(0) = h.L.cy, out.V(0) = cv, out.S(1) = h.Lcrs));
    WSYNC();
    return carry;
}

// lds: WaveLds<N>::NUMS numbers of this wave's LDS (in a host build, windows
// of NLANES E + 9 points and staging of 2 E NLANES slots).
// With SC (rho given) the result is SCALE(MERGE(F, G), rho) in one pass; a
// scaled result that collapses to a line returns 0 (the caller then merges
// and scales in two passes).
// With VO the merge only decides: out receives, per emitted point p >=
// keepL, the record merge_settle describes (F count at X(p), G count at V(p),
// flags at S(p + 1)); S(0) and a kept left crossing are not written, and a
// result without points returns 0.
template <int OP, typename N, bool SC = false, bool VO = false, typename FF, typename GG>
BTD int wave_merge(const FF &F, const GG &G, const Arr<N> &out, N *lds, const N &rho = N{})
{
    if (out.cap < 1) return -1;
    const MergeHead<OP, N> h = merge_head<OP, N, SC>(F, G, rho);
    double pend;
    const int carry = merge_tiles<OP, N, SC, VO>(F, G, out, lds, rho, 0, F.m + G.m, 0, h.keepL, h.psl, &pend, nullptr);
    if (carry < 0) return -1;
    return merge_finish<OP, N, SC, VO>(h, carry, out, rho);
}

// MERGE(F, G, op) of a one-point F when G is strictly better than F at
// every union point (G's points and F's point) and both tails stay with G
// without a crossing (the decisions slot_left and slot_right would take).
// Then every interval keeps G's slope, F's point is dropped by CANON unless
// it equals a point of G (whose abscissa the merge then takes from F), and
// the output is G's points with the values the merge evaluates.  The pass
// writes that output into out while it checks the conditions; it returns
// the count, or -1 when a condition fails (out is then to be overwritten by
// the full merge).  A line G is left to the full merge.
// merge_point_range: the checks and the output of G's points [jb, je);
// returns the count of failed checks over the wave.
template <int OP, typename N>
BTD int merge_point_range(const View<N> &F, const View<N> &G, const Arr<N> &out, int jb, int je)
{
    const int m = G.m;
    // F's one point and slopes, read once; EVAL of F (i = 0 or 1 points of F
    // at or left of y) and of G's piece after x_j (i = j + 1) written out as
    // eval_at computes them
    const N xF = F.X(0), vF = F.V(0), sFa = F.S(0), sFb = F.S(1);
    const double xf = val(xF);
    const auto evalF = [&](int i, const N &y) -> N { return vF + (i ? sFb : sFa) * (y - xF); };
    LV<int> bad;
    LANES(l) {
        int nb = 0;
        // U points of G per lane loaded before any of them is written
        constexpr int U = sizeof(N) == sizeof(double) ? 4 : 1;
        for (int j0 = jb + l; j0 < je; j0 += U * NLANES) {
            N gx[U], gv[U], gs[U];
            double gx1[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = j0 + u * NLANES;
                if (j < je) {
                    gx[u] = G.X(j);
                    gv[u] = G.V(j);
                    gs[u] = G.S(j + 1);
                    gx1[u] = j + 1 < m ? val(G.X(j + 1)) : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = j0 + u * NLANES;
                if (j < je) {
                    const N xj = gx[u];
                    const bool dup = val(xj) == xf;
                    const N P = dup ? xF : xj;
                    // union point P: #{F points <= P} = [P >= x_F], #{G points <= P} = j + 1
                    const N fF = evalF(val(P) >= xf ? 1 : 0, P);
                    const N fG = gv[u] + gs[u] * (P - gx[u]);
                    if (better<OP>(val(fF) - val(fG)) != PG) nb++;
                    out.X(j) = P;
                    out.V(j) = fG;
                    out.S(j + 1) = gs[u];
                    // F's point inside G's piece after x_j
                    if (val(xj) < xf && (j + 1 == m || gx1[u] > xf)) {
                        const N gF = evalF(1, xF), gG = gv[u] + gs[u] * (xF - gx[u]);
                        if (better<OP>(val(gF) - val(gG)) != PG) nb++;
                    }
                }
            }
        }
        bad(l) = nb;
    }
    return lv_exscan(bad);
}

// The checks of that merge that do not belong to one of G's points: the
// capacity, a line G and the tails (*ok false when one fails), and F's point
// left of every point of G (the returned count of failed checks).
template <int OP, typename N>
BTD int wave_merge_point_head(const View<N> &F, const View<N> &G, const Arr<N> &out, bool *ok)
{
    const int m = G.m;
    *ok = false;
    if (out.cap < m || (m == 1 && val(G.S(0)) == val(G.S(1)))) return 0;
    const double sF0 = val(F.S(0)), sG0 = val(G.S(0)), sF1 = val(F.S(1)), sGm = val(G.S(m));
    const bool tails = OP == OPMAX ? (sF0 >= sG0 && sF1 <= sGm) : (sF0 <= sG0 && sF1 >= sGm);
    if (!tails) return 0;
    *ok = true;
    // F's point before every point of G
    const N xF = F.X(0);
    int nb = 0;
    if (val(xF) < val(G.X(0))) {
        const N gF = eval_at<N>(F, 1, xF), gG = eval_at<N>(G, 0, xF);
        if (better<OP>(val(gF) - val(gG)) != PG) nb++;
    }
    return nb;
}

template <int OP, typename N>
BTD int wave_merge_point(const View<N> &F, const View<N> &G, const Arr<N> &out)
{
    bool ok;
    const int nb0 = wave_merge_point_head<OP, N>(F, G, out, &ok);
    if (!ok) return -1;
    const int m = G.m;
    const int nb = nb0 + merge_point_range<OP, N>(F, G, out, 0, m);
    LANE0(out.S(0) = G.S(0));
    WSYNC();
    return nb == 0 ? m : -1;
}

// SCALE by rho from A into out (then CANON).
template <typename N>
BTD int wave_scale(const Arr<N> &A, int m, const N &rho, const Arr<N> &out)
{
    return wave_canon<N>(ScaleSrc<N>{A.view(m), rho}, m, out);
}

// CLIP(A, a, b) into out (seller).
template <typename N>
BTD int wave_clip(const Arr<N> &A, int m, const N &a, const N &b, const Arr<N> &out)
{
    if (val(a) == val(b)) {
        if (out.cap < 1) return -1;
        // i0 = min{j in [0, m] : s[j] >= a}
        LV<int> f;
        LANES(l) {
            int r = m + 1;
            for (int j = l; j <= m; j += NLANES)
                if (val(A.S(j)) >= val(a)) { r = j; break; }
            f(l) = r;
        }
        const int i0 = lv_min_int(f);
        int q = i0 - 1;
        if (q < 0) q = 0;
        if (q > m - 1) q = m - 1;
        LANE0((out.X(0) = A.X(q), out.V(0) = A.V(q), out.S(0) = a, out.S(1) = a));
        WSYNC();
        return 1;
    }
    return wave_canon<N>(ClampSrc<N>{A.view(m), a, b}, m, out);
}

// ---------------------------------------------------------------------------
// The buying half of ENV (same definition as sweep_a).
// h_j = V_j - a X_j; SM_j, Q_j = the minimum of h over i >= j and the
// smallest index attaining it.  Piece j (j < m - 1) leaves x_j with slope
// s_{j+1} (FOLLOW) or a (FLAT), or splits at y_j (SPLIT: s_{j+1} up to y_j,
// then a); the last piece keeps the right tail s_m.  The points of piece j
// depend on the slope arriving at x_j, i.e. on piece j - 1 (a for j = 0).
// ---------------------------------------------------------------------------

template <typename N>
struct SweepElem {
    N rs, y, yv;
    bool sp, fw;   // split; rs is s_{j+1} (FOLLOW or SPLIT) rather than a
};

// Piece j from x_j, v_j, s_{j+1}, x_{j+1} and (SMn, Qn) = (SM_{j+1}, Q_{j+1}).
template <bool MIR, typename N>
BTD SweepElem<N> sweep_elem(const Src<MIR, N> &f, const N &a, int j, int m, const N &xj, const N &vj,
                            const N &spj, const N &xj1, double SMn, int Qn)
{
    SweepElem<N> e;
    e.sp = false;
    e.fw = true;
    e.y = mk<N>(0.0);
    e.yv = mk<N>(0.0);
    if (j == m - 1) {
        e.rs = spj;
        return e;
    }
    int kind = 0;
    const N hj = vj - a * xj;
    if (Qn == j + 1) {
        if (val(spj) >= val(a)) kind = 1;
    } else if (val(hj) < SMn && val(spj) > val(a)) {
        const N xq = f.X(Qn), vq = f.V(Qn);
        const N hq = vq - a * xq;
        const N yy = xj + (hq - hj) / (spj - a);
        if (!(val(yy) < val(xj1))) {
            kind = 1;
        } else if (val(yy) > val(xj)) {
            kind = 2;
            e.y = yy;
            e.yv = vq + a * (yy - xq);
        }
    }
    e.rs = kind != 0 ? spj : a;
    e.fw = kind != 0;
    e.sp = kind == 2;
    return e;
}

// Writes the buying half of ENV of F into out, packed against the right end
// of the buffer: the result is at offset *off (points [*off, *off + count),
// slopes [*off, *off + count]).  Returns the count or -1 on overflow.
// codes (m ints, global memory): for every piece j, bit 0 = the point x_j is
// emitted, bit 1 = the split point y_j is emitted, bit 2 = the slope leaving
// x_j is s_{j+1} (else a).  *line: the result is the one-point line that no
// piece emits.  With VO (decisions only) nothing is written to out (only its
// capacity counts) and qarr[j] receives, for every emitted split point, the
// index of the minimiser it was computed from: wave_sweep_fill then writes
// the points (dual numbers take their decisions on the values this way).
template <bool MIR, typename N, bool VO = false>
BTD int wave_sweep_a(const View<N> &F, const N &a, const Arr<N> &out, int *off, int *codes, bool *line,
                     int *qarr = nullptr)
{
    BT_GLOBAL int *const gcodes = (BT_GLOBAL int *)codes;
    BT_GLOBAL int *const gq = (BT_GLOBAL int *)qarr;
    *line = false;
    constexpr int E = TileE<N>::E;
    struct St {
        N x[E], v[E], s1[E], x1[E], rs[E], y[E], yv[E];
        double h[E];
        int qq[E];
        bool sp[E], fw[E];
    };
    const Src<MIR, N> f{F, F.m};
    const int m = F.m, tm = NLANES * E, cap = out.cap;
    const double av = val(a);
    if (cap < 1) return -1;
    // minimum of h over the tiles already done, on the right
    double SMc = __builtin_huge_val();
    int Qc = 0x7fffffff;
    // the first piece of the tile on the right, settled by the next tile
    bool havep = false, p_sp = false, p_fw = false;
    int p_q = 0;
    N p_x = mk<N>(0.0), p_v = mk<N>(0.0), p_rs = mk<N>(0.0), p_y = mk<N>(0.0), p_yv = mk<N>(0.0);
    int rc = 0;   // points written so far, from the right end
    for (int t1 = m; t1 > 0; t1 -= tm) {
        const int t0 = t1 - tm > 0 ? t1 - tm : 0;
        LV<St> st;
        LV<double> hm;
        LV<int> qm;
        LANES(l) {
            St &q = st(l);
            const int j0 = t0 + l * E;
#pragma unroll
            for (int u = 0; u < E; u++) {
                const int j = j0 + u;
                if (j < t1) {
                    q.x[u] = f.X(j);
                    q.v[u] = f.V(j);
                    q.s1[u] = f.S(j + 1);
                    q.x1[u] = j + 1 < m ? f.X(j + 1) : mk<N>(0.0);
                }
            }
            double hmin = __builtin_huge_val();
            int qmin = 0x7fffffff;
#pragma unroll
            for (int u = E - 1; u >= 0; u--) {
                const int j = j0 + u;
                if (j < t1) {
                    q.h[u] = val(q.v[u] - a * q.x[u]);
                    if (q.h[u] <= hmin) { hmin = q.h[u]; qmin = j; }
                }
            }
            hm(l) = hmin;
            qm(l) = qmin;
        }
        lv_rexmin(hm, qm);
        LV<double> lastc;
        LANES(l) {
            St &q = st(l);
            const int j0 = t0 + l * E;
            double SM = hm(l);
            int Q = qm(l);
            argmin_pick(SM, Q, SMc, Qc);
            double lc = av;
#pragma unroll
            for (int u = E - 1; u >= 0; u--) {
                const int j = j0 + u;
                if (j < t1) {
                    const SweepElem<N> e = sweep_elem<MIR, N>(f, a, j, m, q.x[u], q.v[u], q.s1[u], q.x1[u], SM, Q);
                    q.rs[u] = e.rs; q.y[u] = e.y; q.yv[u] = e.yv; q.sp[u] = e.sp; q.fw[u] = e.fw; q.qq[u] = Q;
                    if (q.h[u] <= SM) { SM = q.h[u]; Q = j; }
                }
            }
            // what the lane's last piece leaves to its right neighbour
#pragma unroll
            for (int u = 0; u < E; u++)
                if (j0 + u < t1) lc = q.sp[u] ? av : val(q.rs[u]);
            lastc(l) = lc;
            hm(l) = SM;
            qm(l) = Q;
        }
        // minimum over i >= t0 (lane 0 holds element t0)
        const double SMn = from_lane<double>(0, [&](int l) { return hm(l); });
        const int Qn = from_lane<int>(0, [&](int l) { return qm(l); });
        // the pending piece t1 settles with the contribution of piece t1 - 1
        const int lt = (t1 - 1 - t0) / E;
        const double cl = from_lane<double>(lt, [&](int l) { return lastc(l); });
        int pc1 = 0, pc2 = 0;
        if (havep) {
            pc1 = cl != val(p_rs) ? 1 : 0;
            pc2 = (p_sp && val(p_rs) != av) ? 1 : 0;
        }
        lv_up1(lastc, av);
        LV<int> c;
        LANES(l) {
            const St &q = st(l);
            const int j0 = t0 + l * E;
            int cc = 0;
#pragma unroll
            for (int u = 0; u < E; u++) {
                const int j = j0 + u;
                if (j < t1 && !(j == t0 && t0 > 0)) {
                    const double sl = j == 0 ? av : (u == 0 ? lastc(l) : (q.sp[u - 1] ? av : val(q.rs[u - 1])));
                    cc += (sl != val(q.rs[u]) ? 1 : 0) + ((q.sp[u] && val(q.rs[u]) != av) ? 1 : 0);
                }
            }
            c(l) = cc;
        }
        const int tot = lv_rexscan(c);
        if (rc + pc1 + pc2 + tot > cap) return -1;
        if (havep) {
            LANE0({
                if constexpr (!VO) {
                    int s = cap - (rc + pc1 + pc2);
                    if (pc1) { out.X(s) = p_x; out.V(s) = p_v; out.S(s + 1) = p_rs; s++; }
                    if (pc2) { out.X(s) = p_y; out.V(s) = p_yv; out.S(s + 1) = a; }
                } else {
                    if (pc2) gq[t1] = p_q;
                }
                gcodes[t1] = pc1 | (pc2 << 1) | (p_fw ? 4 : 0);
            });
        }
        LANES(l) {
            const St &q = st(l);
            const int j0 = t0 + l * E;
            int r = rc + pc1 + pc2 + c(l);   // points to the right of this lane's
#pragma unroll
            for (int u = E - 1; u >= 0; u--) {
                const int j = j0 + u;
                if (j < t1 && !(j == t0 && t0 > 0)) {
                    const double sl = j == 0 ? av : (u == 0 ? lastc(l) : (q.sp[u - 1] ? av : val(q.rs[u - 1])));
                    const int c1 = sl != val(q.rs[u]) ? 1 : 0;
                    const int c2 = (q.sp[u] && val(q.rs[u]) != av) ? 1 : 0;
                    r += c1 + c2;
                    if constexpr (!VO) {
                        int s = cap - r;
                        if (c1) { out.X(s) = q.x[u]; out.V(s) = q.v[u]; out.S(s + 1) = q.rs[u]; s++; }
                        if (c2) { out.X(s) = q.y[u]; out.V(s) = q.yv[u]; out.S(s + 1) = a; }
                    } else {
                        if (c2) gq[j] = q.qq[u];
                    }
                    gcodes[j] = c1 | (c2 << 1) | (q.fw[u] ? 4 : 0);
                }
            }
        }
        rc += pc1 + pc2 + tot;
        SMc = SMn;
        Qc = Qn;
        havep = t0 > 0;
        if (havep) {
            p_x = from_lane<N>(0, [&](int l) { return st(l).x[0]; });
            p_v = from_lane<N>(0, [&](int l) { return st(l).v[0]; });
            p_rs = from_lane<N>(0, [&](int l) { return st(l).rs[0]; });
            p_y = from_lane<N>(0, [&](int l) { return st(l).y[0]; });
            p_yv = from_lane<N>(0, [&](int l) { return st(l).yv[0]; });
            p_sp = from_lane<int>(0, [&](int l) { return st(l).sp[0] ? 1 : 0; }) != 0;
            p_fw = from_lane<int>(0, [&](int l) { return st(l).fw[0] ? 1 : 0; }) != 0;
            p_q = from_lane<int>(0, [&](int l) { return st(l).qq[0]; });
        }
    }
    if (rc == 0) {
        if constexpr (!VO) LANE0((out.X(cap - 1) = f.X(0), out.V(cap - 1) = f.V(0), out.S(cap - 1) = a, out.S(cap) = a));
        *off = cap - 1;
        *line = true;
        WSYNC();
        return 1;
    }
    if constexpr (!VO) LANE0(out.S(cap - rc) = a);
    *off = cap - rc;
    WSYNC();
    return rc;
}

// Writes the points of a sweep whose decisions a VO pass took (codes, qarr;
// rc points, or the one-point line when line): piece j's points go to the
// slots right after those of the pieces before it, packed against the right
// end of out as the sweep itself would have written them, with the same
// arithmetic (x_j, v_j and the slope are copies; a split point is computed
// from x_j, v_j, s_{j+1} and the minimiser's x and v as in sweep_elem).
template <bool MIR, typename N>
BTD void wave_sweep_fill(const View<N> &F, const N &a, const int *codes, const int *qarr, int rc, bool line,
                         const Arr<N> &out)
{
    constexpr int E = 2;
    const BT_GLOBAL int *gcodes = (const BT_GLOBAL int *)codes;
    const BT_GLOBAL int *gq = (const BT_GLOBAL int *)qarr;
    const Src<MIR, N> f{F, F.m};
    const int m = F.m, tm = NLANES * E, cap = out.cap;
    if (line) {
        LANE0((out.X(cap - 1) = f.X(0), out.V(cap - 1) = f.V(0), out.S(cap - 1) = a, out.S(cap) = a));
        WSYNC();
        return;
    }
    int carry = 0;   // points of the pieces already done, on the right
    for (int t1 = m; t1 > 0; t1 -= tm) {
        const int t0 = t1 - tm > 0 ? t1 - tm : 0;
        LV<int> cnt;
        LV<int> cd[E];
        LANES(l) {
            int n = 0;
#pragma unroll
            for (int u = 0; u < E; u++) {
                const int j = t0 + l * E + u;
                const int c = j < t1 ? gcodes[j] : 0;
                cd[u](l) = c;
                n += (c & 1) + ((c >> 1) & 1);
            }
            cnt(l) = n;
        }
        const int tot = lv_rexscan(cnt);
        LANES(l) {
            // slot of the first point of the lane's first piece
            int s = cap - (carry + cnt(l));
#pragma unroll
            for (int u = 0; u < E; u++) s -= (cd[u](l) & 1) + ((cd[u](l) >> 1) & 1);
#pragma unroll
            for (int u = 0; u < E; u++) {
                const int j = t0 + l * E + u;
                const int c = cd[u](l);
                if (c & 3) {
                    const N xj = f.X(j), vj = f.V(j);
                    const N spj = f.S(j + 1);
                    if (c & 1) {
                        out.X(s) = xj; out.V(s) = vj; out.S(s + 1) = (c & 4) ? spj : a;
                        s++;
                    }
                    if (c & 2) {
                        const int Q = gq[j];
                        const N xq = f.X(Q), vq = f.V(Q);
                        const N hj = vj - a * xj;
                        const N hq = vq - a * xq;
                        const N yy = xj + (hq - hj) / (spj - a);
                        out.X(s) = yy; out.V(s) = vq + a * (yy - xq); out.S(s + 1) = a;
                        s++;
                    }
                }
            }
        }
        carry += tot;
    }
    LANE0(out.S(cap - rc) = a);
    WSYNC();
}

// ---------------------------------------------------------------------------
// MERGE_MIN(A, B) of the envelope's two halves without a merge-path search.
// Every point of A and of B = mirror(RB) lies in some interval [x_j, x_j+1)
// of F: at x_j itself, or strictly inside (a split point).  A's points of
// interval j come from piece j of A's sweep, B's from pieces m-1-j (the point
// x_j) and m-2-j (the split inside) of RB's sweep.  The merged order is
// therefore interval by interval: x_j (A's first when both have it, B's then
// being a duplicate), then the split points in increasing order (A's first on
// a tie).  The schedule lists, for every merged position, the point counts of
// A and B after it and whether it starts a union point from A (1), from B (2)
// or not (0: a duplicate), exactly as the merge-path walk records them.
// ---------------------------------------------------------------------------

// Builds the schedule (sF[d] = 4 iF + src, sG[d] = iG for merged positions d
// of the ma + mb points) of pieces [j0, j1) (j0 a multiple of the tile of
// 4 NLANES pieces) from the carries *cAio, *cBio (the point counts of A and
// of B before j0), which it advances to j1.
template <typename N, typename FA, typename FB>
BTD void env_schedule_range(const FA &A, const FB &B, int ma, int mb, const int *codesA, const int *codesR, int m,
                            int *sF, int *sG, int j0, int j1, int *cAio, int *cBio)
{
    constexpr int ES = 4;
    const BT_GLOBAL int *cA = (const BT_GLOBAL int *)codesA;
    const BT_GLOBAL int *cR = (const BT_GLOBAL int *)codesR;
    BT_GLOBAL int *gF = (BT_GLOBAL int *)sF;
    BT_GLOBAL int *gG = (BT_GLOBAL int *)sG;
    int carryA = *cAio, carryB = *cBio;
    for (int t0 = j0; t0 < j1; t0 += NLANES * ES) {
        LV<int> na, nb;
        LV<int> code[ES];
        LANES(l) {
            int a = 0, b = 0;
#pragma unroll
            for (int u = 0; u < ES; u++) {
                const int j = t0 + l * ES + u;
                int c = 0;
                if (j < j1) {
                    const int ca = cA[j];
                    const int cb1 = cR[m - 1 - j] & 1;
                    const int cb2 = j <= m - 2 ? (cR[m - 2 - j] >> 1) & 1 : 0;
                    c = (ca & 3) | (cb1 << 2) | (cb2 << 3);
                }
                code[u](l) = c;
                a += (c & 1) + ((c >> 1) & 1);
                b += ((c >> 2) & 1) + ((c >> 3) & 1);
            }
            na(l) = a;
            nb(l) = b;
        }
        const int totA = lv_exscan(na), totB = lv_exscan(nb);
        LANES(l) {
            int a = carryA + na(l), b = carryB + nb(l);
#pragma unroll
            for (int u = 0; u < ES; u++) {
                const int c = code[u](l);
                int d = a + b;
                const bool a1 = c & 1, a2 = (c >> 1) & 1, b1 = (c >> 2) & 1, b2 = (c >> 3) & 1;
                // x_j
                if (a1 && b1) {
                    gF[d] = 4 * (a + 1) + 1; gG[d] = b + 1; d++;
                    gF[d] = 4 * (a + 1) + 0; gG[d] = b + 1; d++;
                    a++; b++;
                } else if (a1) {
                    gF[d] = 4 * (a + 1) + 1; gG[d] = b; d++;
                    a++;
                } else if (b1) {
                    gF[d] = 4 * a + 2; gG[d] = b + 1; d++;
                    b++;
                }
                // the split points
                if (a2 && b2) {
                    const double ya = a < ma ? val(A.X(a)) : 0.0, yb = b < mb ? val(B.X(b)) : 0.0;
                    if (ya < yb) {
                        gF[d] = 4 * (a + 1) + 1; gG[d] = b; d++;
                        gF[d] = 4 * (a + 1) + 2; gG[d] = b + 1; d++;
                    } else if (ya == yb) {
                        gF[d] = 4 * (a + 1) + 1; gG[d] = b + 1; d++;
                        gF[d] = 4 * (a + 1) + 0; gG[d] = b + 1; d++;
                    } else {
                        gF[d] = 4 * a + 2; gG[d] = b + 1; d++;
                        gF[d] = 4 * (a + 1) + 1; gG[d] = b + 1; d++;
                    }
                    a++; b++;
                } else if (a2) {
                    gF[d] = 4 * (a + 1) + 1; gG[d] = b; d++;
                    a++;
                } else if (b2) {
                    gF[d] = 4 * a + 2; gG[d] = b + 1; d++;
                    b++;
                }
            }
        }
        carryA += totA;
        carryB += totB;
    }
    WSYNC();
    *cAio = carryA;
    *cBio = carryB;
}

// The point counts of A and of B that pieces [0, j1) contribute (the carries
// at j1 of the schedule), from the sweeps' codes.
BTD void env_schedule_carry(const int *codesA, const int *codesR, int m, int j1, int *ca, int *cb)
{
    const BT_GLOBAL int *cA = (const BT_GLOBAL int *)codesA;
    const BT_GLOBAL int *cR = (const BT_GLOBAL int *)codesR;
    LV<int> na, nb;
    LANES(l) {
        int a = 0, b = 0;
        for (int j = l; j < j1; j += NLANES) {
            const int c = cA[j];
            a += (c & 1) + ((c >> 1) & 1);
            b += (cR[m - 1 - j] & 1) + (j <= m - 2 ? (cR[m - 2 - j] >> 1) & 1 : 0);
        }
        na(l) = a;
        nb(l) = b;
    }
    *ca = lv_exscan(na);
    *cb = lv_exscan(nb);
}

// The whole schedule; false when the counts do not add up.
template <typename N, typename FA, typename FB>
BTD bool env_schedule(const FA &A, const FB &B, int ma, int mb, const int *codesA, const int *codesR, int m,
                      int *sF, int *sG)
{
    int ca = 0, cb = 0;
    env_schedule_range<N>(A, B, ma, mb, codesA, codesR, m, sF, sG, 0, m, &ca, &cb);
    return ca == ma && cb == mb;
}

// Merged positions [r0, r1) of MERGE(F, G, op) driven by a schedule (r0 a
// multiple of the tile), emitted into out from position `carry`.  psl: the
// slope arriving at the range's first union point, or NaN when it is not
// known yet: the first union point is then kept, and *first_rs receives the
// slope it leaves (NaN when lane 0 of the first tile starts no union point),
// so that the caller can drop it once the slope arriving there is known.
// Returns the count after the range or -1 on overflow; *psl_out: the slope
// leaving the range.
template <int OP, typename N, typename FF, typename GG>
BTD int merge_sched_tiles(const FF &F, const GG &G, const int *sF, const int *sG, int Lt, int r0, int r1,
                          const Arr<N> &out, N *lds, int carry, double psl, double *psl_out, double *first_rs)
{
    constexpr int E = WaveLds<N>::E;
    constexpr int K = E + 2;
    const BT_GLOBAL int *gF = (const BT_GLOBAL int *)sF;
    const BT_GLOBAL int *gG = (const BT_GLOBAL int *)sG;
    const int tm = NLANES * E;
    const int SZ = 2 * E * NLANES;
    N *stg = lds;
    if (first_rs) *first_rs = __builtin_nan("");
    for (int dt = r0; dt < r1; dt += tm) {
        WSYNC();   // the previous tile's reads of the staging are done
        const int dend = dt + tm < r1 ? dt + tm : r1;
        LV<LaneWalk<E>> wk;
        LANES(l) {
            LaneWalk<E> &w = wk(l);
            const int d0 = dt + l * E;
            const int d1 = d0 + E < dend ? d0 + E : dend;
            w.d0 = d0;
            w.d1 = d1;
            w.pe = d1 + 2 < Lt ? d1 + 2 : Lt;
            w.aend = 0;
            int pf = 0, pg = 0;
#pragma unroll
            for (int k = 0; k < K; k++) {
                int f = pf, g = pg, sc = 0;
                if (d0 < d1 && d0 + k < w.pe) {
                    const int e = gF[d0 + k];
                    f = e >> 2;
                    sc = e & 3;
                    g = gG[d0 + k];
                }
                w.iF[k] = f;
                w.iG[k] = g;
                w.src[k] = sc;
                pf = f;
                pg = g;
            }
        }
        LV<int> c, own;
        LV<double> pso;
        LV<LaneFirst<N>> fst;
        LANES(l) {
            double po;
            own(l) = merge_settle<OP, E, false, N>(F, G, wk(l), stg + l, stg + SZ + l, stg + 2 * SZ + l, NLANES,
                                                   &fst(l), &po, N{});
            pso(l) = po;
        }
        if (first_rs && dt == r0)
            *first_rs = from_lane<double>(0, [&](int l) { return fst(l).have ? val(fst(l).rs) : __builtin_nan(""); });
        const double pnext = from_lane<double>(NLANES - 1, [&](int l) { return pso(l); });
        lv_up1(pso, psl);
        LANES(l) {
            const LaneFirst<N> &f = fst(l);
            const int cf = f.have ? (pso(l) != val(f.rs) ? 1 : 0) + ((f.hc && val(f.rs) != val(f.crs)) ? 1 : 0) : 0;
            c(l) = cf + own(l);
        }
        const int tot = lv_exscan(c);
        if (carry + tot > out.cap) return -1;
        LANES(l) {
            const LaneFirst<N> &f = fst(l);
            int p = carry + c(l);
            if (f.have) {
                if (pso(l) != val(f.rs)) { out.X(p) = f.x; out.V(p) = f.v; out.S(p + 1) = f.rs; p++; }
                if (f.hc && val(f.rs) != val(f.crs)) { out.X(p) = f.cy; out.V(p) = f.cv; out.S(p + 1) = f.crs; p++; }
            }
            const int n = own(l);
#pragma unroll
            for (int k = 0; k < 2 * E; k++) {
                if (k < n) {
                    const int q = k * NLANES + l;
                    out.X(p + k) = stg[q]; out.V(p + k) = stg[SZ + q]; out.S(p + k + 1) = stg[2 * SZ + q];
                }
            }
        }
        carry += tot;
        psl = pnext;
    }
    *psl_out = psl;
    return carry;
}

// The left end of a scheduled merge: its first union point P0, the decision
// there, and the slope arriving at the first tile.
template <int OP, typename N>
struct SchedHead {
    N P0, fF0, fG0;
    Slot<N> L;
    int keepL;
    double psl;
};

template <int OP, typename N, typename FF, typename GG>
BTD SchedHead<OP, N> sched_head(const FF &F, const GG &G)
{
    SchedHead<OP, N> h;
    int iF0, iG0;
    const double xa = val(F.X(0)), xb = val(G.X(0));
    if (xa < xb) { h.P0 = F.X(0); iF0 = 1; iG0 = 0; }
    else if (xb < xa) { h.P0 = G.X(0); iF0 = 0; iG0 = 1; }
    else { h.P0 = F.X(0); iF0 = 1; iG0 = 1; }
    h.fF0 = eval_at<N>(F, iF0, h.P0);
    h.fG0 = eval_at<N>(G, iG0, h.P0);
    h.L = slot_left<OP, N>(F, G, h.P0, h.fF0, h.fG0);
    h.keepL = (h.L.hc && val(h.L.rs) != val(h.L.crs)) ? 1 : 0;
    h.psl = val(h.L.hc ? h.L.crs : h.L.rs);
    return h;
}

// Completes a scheduled merge whose tiles emitted `carry` points.
template <int OP, typename N>
BTD int sched_finish(const SchedHead<OP, N> &h, int carry, const Arr<N> &out)
{
    if (carry == 0) {
        LANE0((out.X(0) = h.L.hc ? h.L.cy : h.P0, out.V(0) = h.L.hc ? h.L.cv : pick<OP, N>(h.fF0, h.fG0),
               out.S(0) = h.L.rs, out.S(1) = h.L.rs));
        WSYNC();
        return 1;
    }
    LANE0(out.S(0) = h.L.rs);
    if (h.keepL) LANE0((out.X(0) = h.L.cy, out.V(0) = h.L.cv, out.S(1) = h.L.crs));
    WSYNC();
    return carry;
}

// MERGE(F, G, op) driven by a schedule instead of the merge-path walk (same
// result as wave_merge); F and G are read from global memory, LDS holds only
// the staging of the emitted points.
template <int OP, typename N, typename FF, typename GG>
BTD int wave_merge_sched(const FF &F, const GG &G, const int *sF, const int *sG, const Arr<N> &out, N *lds)
{
    if (out.cap < 1) return -1;
    const SchedHead<OP, N> h = sched_head<OP, N>(F, G);
    double pend;
    const int carry = merge_sched_tiles<OP, N>(F, G, sF, sG, F.m + G.m, 0, F.m + G.m, out, lds, h.keepL, h.psl,
                                               &pend, nullptr);
    if (carry < 0) return -1;
    return sched_finish<OP, N>(h, carry, out);
}

// ---------------------------------------------------------------------------
// Dual numbers: the first MERGE of a node update takes its decisions on the
// values (a binary64 merge over value views, in decisions-only mode) and then
// rebuilds every emitted point with its tangents from the recorded pieces,
// with the settle step's own arithmetic; the records are independent, so the
// rebuild runs several points per lane at once.  (For the envelope's
// MERGE_MIN the rebuild measured slower than the dual-number merge itself.)
// ---------------------------------------------------------------------------

// The value parts of a function of dual numbers, as a binary64 function.
BTD View<double> vview(const View<D4> &f)
{
    constexpr int NT = (int)(sizeof(D4) / sizeof(double));
    return View<double>{(const double *)f.x, (const double *)f.v, (const double *)f.s, f.m, NT * f.st};
}

// Points [p0, n) of out from their records (merge_settle, VO).
template <int OP, bool SC, typename N, typename FF, typename GG>
BTD void merge_fill(const FF &F, const GG &G, const Arr<double> &rec, int p0, int n, const Arr<N> &out,
                    const N &rho)
{
    constexpr int U = 4;   // records per lane per step, their loads issued together
    LANES(l) {
        for (int p1 = p0 + l; p1 < n; p1 += U * NLANES) {
            int iF[U], iG[U], fl[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int p = p1 + u * NLANES;
                const int q = p < n ? p : p1;
                iF[u] = (int)rec.X(q); iG[u] = (int)rec.V(q); fl[u] = (int)rec.S(q + 1);
            }
            Seg<N> gF[U], gG[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                gF[u] = seg_at<N>(F, iF[u]);
                gG[u] = seg_at<N>(G, iG[u]);
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int p = p1 + u * NLANES;
                if (p < n) {
                    const N P = (fl[u] & 2) ? gF[u].x : gG[u].x;
                    const N fF = seg_eval<N>(gF[u], P), fG = seg_eval<N>(gG[u], P);
                    N x, v;
                    if (fl[u] & 1) {
                        x = P + (fF - fG) / (gG[u].s - gF[u].s);
                        v = (fl[u] & 4) ? seg_eval<N>(gF[u], x) : seg_eval<N>(gG[u], x);
                    } else {
                        x = P;
                        v = (fl[u] & 4) ? fF : fG;
                    }
                    N sl = (fl[u] & 8) ? gF[u].s : gG[u].s;
                    if constexpr (SC) {
                        v = v * rho;
                        sl = sl * rho;
                    }
                    out.X(p) = x; out.V(p) = v; out.S(p + 1) = sl;
                }
            }
        }
    }
    WSYNC();
}

// The left tail of MERGE(F, G): S(0) and a kept crossing before the first
// union point, written as wave_merge writes them; returns keepL.
template <int OP, bool SC, typename N, typename FF, typename GG>
BTD int merge_left_write(const FF &F, const GG &G, const Arr<N> &out, const N &rho)
{
    const auto scl = [&](const N &x) -> N {
        if constexpr (SC) return x * rho;
        else return x;
    };
    N P0;
    int iF0, iG0;
    {
        const double xa = val(F.X(0)), xb = val(G.X(0));
        if (xa < xb) { P0 = F.X(0); iF0 = 1; iG0 = 0; }
        else if (xb < xa) { P0 = G.X(0); iF0 = 0; iG0 = 1; }
        else { P0 = F.X(0); iF0 = 1; iG0 = 1; }
    }
    const N fF0 = eval_at<N>(F, iF0, P0), fG0 = eval_at<N>(G, iG0, P0);
    const Slot<N> L = slot_left<OP, N>(F, G, P0, fF0, fG0);
    const N Lrs = scl(L.rs), Lcrs = L.hc ? scl(L.crs) : Lrs;
    const int keepL = (L.hc && val(Lrs) != val(Lcrs)) ? 1 : 0;
    LANE0(out.S(0) = Lrs);
    if (keepL) LANE0((out.X(0) = L.cy, out.V(0) = scl(L.cv), out.S(1) = Lcrs));
    return keepL;
}

// wave_merge for dual numbers (same result): decisions on the values, then
// the points.  Falls back to the dual-number merge itself when the records
// find no room or the result has no points.
template <int OP, bool SC, typename FF, typename GG>
BTD int wave_merge_d4(const FF &F, const GG &G, const Arr<D4> &out, D4 *lds, const D4 &rho, WaveTmp &T)
{
    static_assert(WaveLds<double>::NUMS * sizeof(double) <= WaveLds<D4>::NUMS * sizeof(D4),
                  "the binary64 merge must fit the dual-number wave's LDS");
    const int64_t mark = T.used;
    Arr<double> rec;
    int n = 0;
    if (T.arr<double>(out.cap, &rec)) n = wave_merge<OP, double, SC, true>(vview(F), vview(G), rec, (double *)lds, val(rho));
    if (n <= 0) {
        T.used = mark;
        if (n < 0) return -1;
        return wave_merge<OP, D4, SC>(F, G, out, lds, rho);
    }
    const int keepL = merge_left_write<OP, SC, D4>(F, G, out, rho);
    merge_fill<OP, SC, D4>(F, G, rec, keepL, n, out, rho);
    T.used = mark;
    return n;
}

// ENV(F, a, b) into out (buyer).
// A request from the wave that updates a node to another wave of its
// workgroup that has no node of its own left at the level (binary64, device
// builds): a part of the envelope's work that the helper runs while the
// node's own wave runs the rest.  The mailbox lives in LDS; state 0 idle, 1
// request posted, 4 taken by the helper, 2 done, 3 no more requests (the
// node is finished).  A posted request that no helper has taken when the
// node's wave needs its result is taken back (1 -> 0) and run by that wave,
// so neither side ever waits on a wave that is not working for it.
struct SweepHelp {
    int state, kind;             // kind 1: the mirror sweep; 2: the upper half of MERGE_MIN(A, B);
                                 // 3: the upper half of the first MERGE (with SCALE); 4: the
                                 // upper half of the exercise merge's shortcut; 5: the upper half
                                 // of the envelope's schedule
    int m, st, cap;              // 1, 3, 4: F's points and stride; all: the output's capacity
    const double *fx, *fv, *fs;  // 1, 3, 4: F
    const double *gx, *gv, *gs;  // 3, 4: G
    int gm, gst;                 // 3, 4: G's points and stride
    double *ox, *ov, *os;        // both: the output
    int *codes;                  // 1: the sweep's codes; 5: A's sweep codes
    int *codes2;                 // 5: RB's sweep codes
    int *sF2, *sG2;              // 5: the schedule
    double slope;                // 1: the sweep's slope (-b); 3: rho
    const double *ax, *av, *as, *rx, *rv, *rs;   // 2: A and RB (unit stride)
    const int *sF, *sG;          // 2: the schedule
    int ma, mrb, Lt, D;          // 2: point counts; 2, 3: merged positions; 2, 3, 4: first position of the half
    int off, line, count;        // results
    double frs;                  // 2, 3: the slope its first union point leaves
};

#ifndef BT_HOST_DEBUG
// One mailbox per wave of a workgroup (indexed by the requesting wave).
__shared__ SweepHelp bt_help[NWAVE];

__device__ __forceinline__ int help_state(int i)
{
    return __hip_atomic_load(&bt_help[i].state, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void help_post(int i, int st)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (WLANE == 0) __hip_atomic_store(&bt_help[i].state, st, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    wave_sync();
}

// Moves mailbox i from state `from` to `to` if it is in `from` (one lane,
// result shared by the wave).
__device__ __forceinline__ bool help_cas(int i, int from, int to)
{
    int ok = 0;
    if (WLANE == 0) {
        int e = from;
        ok = __hip_atomic_compare_exchange_strong(&bt_help[i].state, &e, to, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP) ? 1 : 0;
    }
    ok = __builtin_amdgcn_readfirstlane(ok);
    wave_sync();
    return ok != 0;
}

// The node's wave, after its own part: takes the request back if no helper
// took it (true: run the helper's part itself), else waits for its result.
__device__ __forceinline__ bool help_reclaim(int i)
{
    if (help_cas(i, 1, 0)) return true;
    while (help_state(i) != 2) __builtin_amdgcn_s_sleep(1);
    return false;
}

// The helper's side: serves the requests of wave i until it posts 3 (lds:
// the helper's own LDS slice).
__device__ __forceinline__ void sweep_helper(int i, double *lds)
{
    SweepHelp *h = &bt_help[i];
    for (;;) {
        int st;
        while ((st = help_state(i)) != 1 && st != 3) __builtin_amdgcn_s_sleep(1);
        if (st == 3) break;
        if (!help_cas(i, 1, 4)) continue;   // taken back meanwhile
        const Arr<double> out{h->ox, h->ov, h->os, 1, h->cap};
        if (h->kind == 1) {
            const View<double> F{h->fx, h->fv, h->fs, h->m, h->st};
            int off = 0;
            bool line = false;
            const int n = wave_sweep_a<true, double>(F, h->slope, out, &off, h->codes, &line);
            if (WLANE == 0) {
                h->off = off;
                h->line = line ? 1 : 0;
                h->count = n;
            }
        } else if (h->kind == 5) {
            const View<double> Av{h->ax, h->av, h->as, h->ma, 1};
            const View<double> Rv{h->rx, h->rv, h->rs, h->mrb, 1};
            const MirSrc<double> Bv{Rv, h->mrb};
            int ca = 0, cb = 0;
            env_schedule_carry(h->codes, h->codes2, h->m, h->D, &ca, &cb);
            env_schedule_range<double>(Av, Bv, h->ma, h->mrb, h->codes, h->codes2, h->m, h->sF2, h->sG2, h->D, h->m,
                                       &ca, &cb);
            if (WLANE == 0) {
                h->count = ca;
                h->off = cb;
            }
        } else if (h->kind == 4) {
            const View<double> F{h->fx, h->fv, h->fs, h->m, h->st}, G{h->gx, h->gv, h->gs, h->gm, h->gst};
            const int n = merge_point_range<OPMIN, double>(F, G, out, h->D, G.m);
            if (WLANE == 0) h->count = n;
        } else if (h->kind == 3) {
            const View<double> F{h->fx, h->fv, h->fs, h->m, h->st}, G{h->gx, h->gv, h->gs, h->gm, h->gst};
            const int D = h->D;
            const int at = merge_path_in(F, G, D, D - G.m > 0 ? D - G.m : 0, D < F.m ? D : F.m);
            double pend, frs;
            const int n = merge_tiles<OPMAX, double, true, false>(F, G, out, (double *)lds, h->slope, D, h->Lt, at,
                                                                  0, __builtin_nan(""), &pend, &frs);
            if (WLANE == 0) {
                h->count = n;
                h->frs = frs;
            }
        } else {
            const View<double> Av{h->ax, h->av, h->as, h->ma, 1};
            const View<double> Rv{h->rx, h->rv, h->rs, h->mrb, 1};
            const MirSrc<double> Bv{Rv, h->mrb};
            double pend, frs;
            const int n = merge_sched_tiles<OPMIN, double>(Av, Bv, h->sF, h->sG, h->Lt, h->D, h->Lt, out, lds, 0,
                                                           __builtin_nan(""), &pend, &frs);
            if (WLANE == 0) {
                h->count = n;
                h->frs = frs;
            }
        }
        help_post(i, 2);
    }
}
#else
inline int bt_host_split = 0;   // host builds: run the split MERGE_MIN(A, B) on one emulated wave
inline long long bt_host_split_stats[2];   // split merges, and first points of an upper half dropped
#endif

// Copies n points (abscissa, value and the slope after each) from src's
// point s0 on to dst's point d0 on, with four points per lane in flight.
BTD void copy_points(const Arr<double> &dst, int d0, const Arr<double> &src, int s0, int n)
{
    constexpr int U = 4;
    LANES(l) {
        for (int i0 = 0; i0 < n; i0 += U * NLANES) {
            double x[U], v[U], sl[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int i = i0 + u * NLANES + l;
                if (i < n) {
                    x[u] = src.X(s0 + i);
                    v[u] = src.V(s0 + i);
                    sl[u] = src.S(s0 + i + 1);
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int i = i0 + u * NLANES + l;
                if (i < n) {
                    dst.X(d0 + i) = x[u];
                    dst.V(d0 + i) = v[u];
                    dst.S(d0 + i + 1) = sl[u];
                }
            }
        }
    }
    WSYNC();
}

// MERGE_MIN(A, B) of the envelope from its schedule, the upper half of its
// merged positions (from a tile boundary) run by the helper wave `help` on
// the GPU, or before the lower half on the same wave in a host build with
// bt_host_split set.  The upper half is emitted into a buffer of its own from
// an unknown arriving slope, so its first union point is kept; the node's
// wave drops it when the slope arriving there (the one its own half leaves)
// equals the slope it leaves -- the decision the whole merge takes there --
// and appends the rest.  Returns -2 when the merge is not split (no helper,
// fewer than four tiles, or no room for the buffer).
BTD int env_merge_split(const View<double> &Av, const View<double> &Rv, const MirSrc<double> &Bv, int ma, int mrb,
                        const int *sF, const int *sG, const Arr<double> &out, double *lds, WaveTmp &T, int help)
{
    const int tm = NLANES * WaveLds<double>::E;
    const int Lt = ma + mrb;
#ifdef BT_HOST_DEBUG
    const bool split = bt_host_split != 0;
    (void)help;
#else
    const bool split = help >= 0;
#endif
    if (!split || Lt < 4 * tm || out.cap < 1) return -2;
    const int D = (Lt / 2 / tm) * tm;
    const int64_t mark = T.used;
    Arr<double> o2;
    if (!T.arr<double>(out.cap, &o2)) return -2;
    int n2;
    double frs;
#ifdef BT_HOST_DEBUG
    {
        double pe2;
        n2 = merge_sched_tiles<OPMIN, double>(Av, Bv, sF, sG, Lt, D, Lt, o2, lds, 0, __builtin_nan(""), &pe2, &frs);
    }
#else
    SweepHelp &h = bt_help[help];
    if (WLANE == 0) {
        h.kind = 2;
        h.ax = Av.x; h.av = Av.v; h.as = Av.s; h.ma = ma;
        h.rx = Rv.x; h.rv = Rv.v; h.rs = Rv.s; h.mrb = mrb;
        h.sF = sF; h.sG = sG; h.Lt = Lt; h.D = D;
        h.ox = o2.x; h.ov = o2.v; h.os = o2.s; h.cap = o2.cap;
    }
    help_post(help, 1);
#endif
    const SchedHead<OPMIN, double> hd = sched_head<OPMIN, double>(Av, Bv);
    double pend;
    const int c1 = merge_sched_tiles<OPMIN, double>(Av, Bv, sF, sG, Lt, 0, D, out, lds, hd.keepL, hd.psl, &pend,
                                                    nullptr);
#ifndef BT_HOST_DEBUG
    if (help_reclaim(help)) {
        double pe2;
        n2 = merge_sched_tiles<OPMIN, double>(Av, Bv, sF, sG, Lt, D, Lt, o2, lds, 0, __builtin_nan(""), &pe2, &frs);
    } else {
        n2 = h.count;
        frs = h.frs;
    }
#endif
    int total = -1;
    if (c1 >= 0 && n2 >= 0) {
        const int drop = frs == pend ? 1 : 0;
#ifdef BT_HOST_DEBUG
        bt_host_split_stats[0]++;
        bt_host_split_stats[1] += drop;
#endif
        if (c1 + n2 - drop <= out.cap) {
            const int n = n2 - drop;
            copy_points(out, c1, o2, drop, n);
            total = sched_finish<OPMIN, double>(hd, c1 + n, out);
        }
    }
    T.used = mark;
    return total;
}

// SCALE(MERGE(Zu, Zd), rho) (the first step of a node update), split as
// env_merge_split splits MERGE_MIN(A, B): the upper half of the merged
// positions (from a tile boundary, with its merge-path coordinate found by
// search) runs on the helper wave, or first on the same wave in a host build
// with bt_host_split set.  Returns -2 when the merge is not split, and as
// wave_merge<OPMAX, double, true> otherwise.
BTD int merge_scale_split(const View<double> &Zu, const View<double> &Zd, const Arr<double> &out, double *lds,
                          double rho, WaveTmp &T, int help)
{
    const int tm = NLANES * WaveLds<double>::E;
    const int Lt = Zu.m + Zd.m;
#ifdef BT_HOST_DEBUG
    const bool split = bt_host_split != 0;
    (void)help;
#else
    const bool split = help >= 0;
#endif
    if (!split || Lt < 4 * tm || out.cap < 1) return -2;
    const int D = (Lt / 2 / tm) * tm;
    const int64_t mark = T.used;
    Arr<double> o2;
    if (!T.arr<double>(out.cap, &o2)) return -2;
    int n2;
    double frs;
#ifdef BT_HOST_DEBUG
    {
        double pe2;
        const int at = merge_path_in(Zu, Zd, D, D - Zd.m > 0 ? D - Zd.m : 0, D < Zu.m ? D : Zu.m);
        n2 = merge_tiles<OPMAX, double, true, false>(Zu, Zd, o2, lds, rho, D, Lt, at, 0, __builtin_nan(""), &pe2,
                                                     &frs);
    }
#else
    SweepHelp &h = bt_help[help];
    if (WLANE == 0) {
        h.kind = 3;
        h.fx = Zu.x; h.fv = Zu.v; h.fs = Zu.s; h.m = Zu.m; h.st = Zu.st;
        h.gx = Zd.x; h.gv = Zd.v; h.gs = Zd.s; h.gm = Zd.m; h.gst = Zd.st;
        h.slope = rho; h.Lt = Lt; h.D = D;
        h.ox = o2.x; h.ov = o2.v; h.os = o2.s; h.cap = o2.cap;
    }
    help_post(help, 1);
#endif
    const MergeHead<OPMAX, double> hd = merge_head<OPMAX, double, true>(Zu, Zd, rho);
    double pend;
    const int c1 = merge_tiles<OPMAX, double, true, false>(Zu, Zd, out, lds, rho, 0, D, 0, hd.keepL, hd.psl, &pend,
                                                           nullptr);
#ifndef BT_HOST_DEBUG
    if (help_reclaim(help)) {
        double pe2;
        const int at = merge_path_in(Zu, Zd, D, D - Zd.m > 0 ? D - Zd.m : 0, D < Zu.m ? D : Zu.m);
        n2 = merge_tiles<OPMAX, double, true, false>(Zu, Zd, o2, lds, rho, D, Lt, at, 0, __builtin_nan(""), &pe2,
                                                     &frs);
    } else {
        n2 = h.count;
        frs = h.frs;
    }
#endif
    int total = -1;
    if (c1 >= 0 && n2 >= 0) {
        const int drop = frs == pend ? 1 : 0;
#ifdef BT_HOST_DEBUG
        bt_host_split_stats[0]++;
        bt_host_split_stats[1] += drop;
#endif
        if (c1 + n2 - drop <= out.cap) {
            const int n = n2 - drop;
            copy_points(out, c1, o2, drop, n);
            total = merge_finish<OPMAX, double, true, false>(hd, c1 + n, out, rho);
        }
    }
    T.used = mark;
    return total;
}

// The envelope's schedule with the pieces from a tile boundary J on built by
// the helper wave, which first counts the points that pieces [0, J)
// contribute; the schedule's positions follow from those counts, so the two
// halves write their own entries.  Returns as env_schedule.
BTD bool env_schedule_split(const View<double> &Av, const View<double> &Rv, const MirSrc<double> &Bv, int ma, int mrb,
                            int *codesA, int *codesR, int m, int *sF, int *sG, int help)
{
#ifdef BT_HOST_DEBUG
    const bool split = bt_host_split != 0;
    (void)help;
#else
    const bool split = help >= 0;
#endif
    const int tile = 4 * NLANES;
    if (!split || m < 4 * tile) return env_schedule<double>(Av, Bv, ma, mrb, codesA, codesR, m, sF, sG);
    const int J = (m / 2 / tile) * tile;
    int ca2 = 0, cb2 = 0;
#ifdef BT_HOST_DEBUG
    env_schedule_carry(codesA, codesR, m, J, &ca2, &cb2);
    env_schedule_range<double>(Av, Bv, ma, mrb, codesA, codesR, m, sF, sG, J, m, &ca2, &cb2);
#else
    SweepHelp &h = bt_help[help];
    if (WLANE == 0) {
        h.kind = 5;
        h.ax = Av.x; h.av = Av.v; h.as = Av.s; h.ma = ma;
        h.rx = Rv.x; h.rv = Rv.v; h.rs = Rv.s; h.mrb = mrb;
        h.codes = codesA; h.codes2 = codesR; h.m = m; h.sF2 = sF; h.sG2 = sG; h.D = J;
    }
    help_post(help, 1);
#endif
    int ca = 0, cb = 0;
    env_schedule_range<double>(Av, Bv, ma, mrb, codesA, codesR, m, sF, sG, 0, J, &ca, &cb);
#ifndef BT_HOST_DEBUG
    if (help_reclaim(help)) {
        ca2 = ca;
        cb2 = cb;
        env_schedule_range<double>(Av, Bv, ma, mrb, codesA, codesR, m, sF, sG, J, m, &ca2, &cb2);
    } else {
        ca2 = h.count;
        cb2 = h.off;
    }
#endif
    return ca2 == ma && cb2 == mrb;
}

// The buyer's exercise merge shortcut (wave_merge_point<OPMIN>) with the
// upper half of V's points checked and written by the helper wave: every
// point's output has a fixed place, so the halves need no joining.  Returns
// -2 when not split, else as wave_merge_point.
BTD int merge_point_split(const View<double> &F, const View<double> &G, const Arr<double> &out, int help)
{
#ifdef BT_HOST_DEBUG
    const bool split = bt_host_split != 0;
    (void)help;
#else
    const bool split = help >= 0;
#endif
    const int m = G.m, uw = 4 * NLANES;
    if (!split || m < 4 * uw) return -2;
    bool ok;
    const int nb0 = wave_merge_point_head<OPMIN, double>(F, G, out, &ok);
    if (!ok) return -1;
    const int J = (m / 2 / uw) * uw;
    int nb2;
#ifdef BT_HOST_DEBUG
    nb2 = merge_point_range<OPMIN, double>(F, G, out, J, m);
#else
    SweepHelp &h = bt_help[help];
    if (WLANE == 0) {
        h.kind = 4;
        h.fx = F.x; h.fv = F.v; h.fs = F.s; h.m = F.m; h.st = F.st;
        h.gx = G.x; h.gv = G.v; h.gs = G.s; h.gm = G.m; h.gst = G.st;
        h.ox = out.x; h.ov = out.v; h.os = out.s; h.cap = out.cap;
        h.D = J;
    }
    help_post(help, 1);
#endif
    const int nb1 = merge_point_range<OPMIN, double>(F, G, out, 0, J);
#ifndef BT_HOST_DEBUG
    if (help_reclaim(help)) nb2 = merge_point_range<OPMIN, double>(F, G, out, J, m);
    else nb2 = h.count;
#endif
    LANE0(out.S(0) = G.S(0));
    WSYNC();
    return nb0 + nb1 + nb2 == 0 ? m : -1;
}

template <typename N>
BTD int wave_env(const Arr<N> &Fa, int m, const N &a, const N &b, const Arr<N> &out, WaveTmp &T, N *lds,
                 int help = -1)
{
    const int64_t mark = T.used;
    const View<N> F = Fa.view(m);
    if (val(a) == val(b)) {
        if (out.cap < 1) return -1;
        // the line of slope a through the first minimiser of V_j - a X_j
        LV<double> h;
        LV<int> q;
        LANES(l) {
            double hb = __builtin_huge_val();
            int qb = 0x7fffffff;
            for (int j = l; j < m; j += NLANES) {
                const double hv = val(F.V(j) - a * F.X(j));
                if (hv < hb) { hb = hv; qb = j; }
            }
            h(l) = hb;
            q(l) = qb;
        }
        const int js = lv_argmin(h, q);
        LANE0((out.X(0) = F.X(js), out.V(0) = F.V(js), out.S(0) = a, out.S(1) = a));
        WSYNC();
        return 1;
    }
    Arr<N> A, RB;
    if (!T.arr<N>(2 * m, &A) || !T.arr<N>(2 * m, &RB)) { T.used = mark; return -1; }
    int *codes = (int *)T.dbl((int64_t)m + 1);   // 2 m ints
    if (!codes) { T.used = mark; return -1; }
    int *codesA = codes, *codesR = codes + m;
    int offA = 0, offR = 0, ma = -1, mrb = -1;
    bool lineA = false, lineR = false;
    if constexpr (sizeof(N) == sizeof(double)) {
#ifndef BT_HOST_DEBUG
        if (help >= 0) {
            // the mirror sweep goes to the helper wave, the direct one stays
            SweepHelp &h = bt_help[help];
            if (WLANE == 0) {
                h.kind = 1;
                h.m = m; h.st = F.st; h.cap = RB.cap;
                h.fx = F.x; h.fv = F.v; h.fs = F.s;
                h.ox = RB.x; h.ov = RB.v; h.os = RB.s;
                h.codes = codesR;
                h.slope = -b;
            }
            help_post(help, 1);
            ma = wave_sweep_a<false, N>(F, a, A, &offA, codesA, &lineA);
            if (help_reclaim(help)) {
                mrb = ma < 0 ? -1 : wave_sweep_a<true, N>(F, -b, RB, &offR, codesR, &lineR);
            } else {
                mrb = ma < 0 ? -1 : h.count;
                offR = h.off;
                lineR = h.line != 0;
            }
        } else
#endif
        {
            ma = wave_sweep_a<false, N>(F, a, A, &offA, codesA, &lineA);
            mrb = ma < 0 ? -1 : wave_sweep_a<true, N>(F, -b, RB, &offR, codesR, &lineR);
        }
    } else {
        // dual numbers: the decisions on the values (a binary64 sweep over
        // the value parts, several pieces per lane), then the points with
        // their tangents
        int *qs = (int *)T.dbl((int64_t)m + 1);   // 2 m ints
        if (!qs) { T.used = mark; return -1; }
        constexpr int NT = (int)(sizeof(N) / sizeof(double));
        const View<double> Fv{(const double *)F.x, (const double *)F.v, (const double *)F.s, m, NT * F.st};
        const Arr<double> capA{nullptr, nullptr, nullptr, 1, A.cap}, capR{nullptr, nullptr, nullptr, 1, RB.cap};
        ma = wave_sweep_a<false, double, true>(Fv, val(a), capA, &offA, codesA, &lineA, qs);
        mrb = ma < 0 ? -1 : wave_sweep_a<true, double, true>(Fv, -val(b), capR, &offR, codesR, &lineR, qs + m);
        if (ma >= 0 && mrb >= 0) {
            wave_sweep_fill<false, N>(F, a, codesA, qs, ma, lineA, A);
            wave_sweep_fill<true, N>(F, -b, codesR, qs + m, mrb, lineR, RB);
        }
    }
    if (ma < 0 || mrb < 0) { T.used = mark; return -1; }
    const View<N> Av{A.x + offA, A.v + offA, A.s + offA, ma, 1};
    const View<N> Rv{RB.x + offR, RB.v + offR, RB.s + offR, mrb, 1};
    // B = CANON(mirror image of RB) is the mirror image itself: the sweep
    // emits a point only where its slope changes (and a one-point line stays
    // one point), so the merge reads RB through the mirror
    const MirSrc<N> Bv{Rv, mrb};
    int mv = -1;
    bool done = false;
    if (!lineA && !lineR) {
        const int64_t nd = ((int64_t)ma + mrb + 2) / 2;   // ma + mrb ints
        int *sF = (int *)T.dbl(nd), *sG = (int *)T.dbl(nd);
        bool sched = false;
        if (sF && sG) {
            if constexpr (sizeof(N) == sizeof(double))
                sched = env_schedule_split(Av, Rv, Bv, ma, mrb, codesA, codesR, m, sF, sG, help);
            else
                sched = env_schedule<N>(Av, Bv, ma, mrb, codesA, codesR, m, sF, sG);
        }
        if (sched) {
            mv = -2;
            if constexpr (sizeof(N) == sizeof(double)) mv = env_merge_split(Av, Rv, Bv, ma, mrb, sF, sG, out, lds, T, help);
            if (mv == -2) mv = wave_merge_sched<OPMIN, N>(Av, Bv, sF, sG, out, lds);
            done = true;
        }
    }
    if (!done) mv = wave_merge<OPMIN, N>(Av, Bv, out, lds);
#ifdef BT_HOST_DEBUG
    bt_host_env_sched[done ? 0 : 1]++;
#endif
    T.used = mark;
    return mv;
}

// One node update by a whole wave (see node_update).  The result is left in
// *zout inside T's slice (valid until T is reset).  lds: this wave's
// WaveLds<N>::NUMS numbers of LDS.  exf: as in node_update.  help (binary64
// buyer, device builds): the mailbox (bt_help index) an idle wave serves for
// this node, or -1.
template <int SIDE, typename N>
BTD int wave_node_update(const View<N> &Zu, const View<N> &Zd, const N &S, const N &kt, const N &rho,
                         const N &xi, const N &zeta, bool exercise, WaveTmp &T, N *lds, Arr<N> *zout,
                         int *exf = nullptr, int help = -1)
{
    const N one = mk<N>(1.0);
    const N a = -((one + kt) * S);
    const N b = -((one - kt) * S);
    const int M = Zu.m + Zd.m;
    Arr<N> W, W2, V;
    if (!T.arr<N>(2 * M + 1, &W)) return -1;
    // f = SCALE(MERGE(Zu, Zd), rho), in one pass unless the result is a line
    int mw;
    if constexpr (sizeof(N) == sizeof(double)) {
        mw = SIDE == 1 ? merge_scale_split(Zu, Zd, W, lds, rho, T, help) : -2;
        if (mw == -2) mw = wave_merge<OPMAX, N, true>(Zu, Zd, W, lds, rho);
    } else {
        mw = wave_merge_d4<OPMAX, true>(Zu, Zd, W, lds, rho, T);
    }
    if (mw == 0) {
        mw = wave_merge<OPMAX, N>(Zu, Zd, W, lds);
        if (mw < 0 || !T.arr<N>(mw, &W2)) return -1;
        mw = wave_scale(W, mw, rho, W2);
        W = W2;
    }
    if (mw < 0) return -1;
    int mv;
    if (SIDE == 0) {
        if (!T.arr<N>(mw, &V)) return -1;
        mv = wave_clip(W, mw, a, b, V);
    } else {
        // the output of ENV is bounded by 8 mw + 1 points but is about mw in
        // practice: try a buffer of 2 mw + 8 first and fall back to the bound
        const int64_t markv = T.used;
        if (!T.arr<N>(2 * mw + 8, &V)) return -1;
        mv = wave_env(W, mw, a, b, V, T, lds, help);
        if (mv < 0) {
            T.used = markv;
            if (!T.arr<N>(8 * mw + 1, &V)) return -1;
            mv = wave_env(W, mw, a, b, V, T, lds, help);
        }
    }
    if (mv < 0) return -1;
    if constexpr (sizeof(N) == sizeof(double)) {
        if (exf) *exf = exercise ? exercise_flag<SIDE, N>(V.view(mv), xi, zeta, a, b) : 0;
    }
    if (!exercise) { *zout = V; return mv; }
    Arr<N> U, Z;
    if (!T.arr<N>(1, &U) || !T.arr<N>(2 * mv + 3, &Z)) return -1;
    LANE0((U.X(0) = SIDE == 0 ? zeta : -zeta, U.V(0) = SIDE == 0 ? xi : -xi, U.S(0) = a, U.S(1) = b));
    WSYNC();
    // no exercise at or near this node: the merge keeps V's points
    int mz = -2;
    if constexpr (SIDE == 1 && sizeof(N) == sizeof(double)) mz = merge_point_split(U.view(1), V.view(mv), Z, help);
    if (mz == -2) mz = wave_merge_point<SIDE == 0 ? OPMAX : OPMIN, N>(U.view(1), V.view(mv), Z);
    if (mz < 0) mz = wave_merge<SIDE == 0 ? OPMAX : OPMIN, N>(U.view(1), V.view(mv), Z, lds);
    *zout = Z;
    return mz;
}

}  // namespace bt
