// bt_device.hpp -- shared definitions of the gfx950 kernels and their host
// launcher: per-option tree constants, the per-lane temporary layout, and
// the per-node update of Section 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BTHD __host__ __device__ inline

#include "bt_model.hpp"
#include "bt_pwl.hpp"

namespace bt {

constexpr int WG = 256;          // lanes per workgroup (4 waves of 64)
constexpr int NWAVE = WG / 64;
constexpr int SMALL_CAP = 12;    // points per stage on the interleaved fast path

enum { PAY_PUT = 0, PAY_CALL = 1, PAY_BULL = 2, PAY_PUT_CASH = 3, PAY_CALL_CASH = 4, PAY_BEAR = 5, PAY_STRADDLE = 6 };
enum { F_EUROPEAN = 1u, F_COST_AT_T0 = 2u };

// The model's inputs as numbers of type T: plain values, or for D4 the
// values with their tangents seeded for (S0, sigma, R, k):
// dS0/dS0 = 1, du/dsigma = u sqrt(T/N), dr/dR = r T/N, dk/dk = 1, and
// d = 1/u, rho = 1/r carried through the division.
template <typename T>
struct Inputs {
    T S0, u, d, rho, k, K, K2;
};

BTD Inputs<double> inputs_of(const Model &md, double)
{
    return Inputs<double>{md.S0, md.u, md.d, md.rho, md.k, md.K, md.K2};
}

BTD Inputs<D4> inputs_of(const Model &md, D4)
{
    Inputs<D4> in;
    in.S0 = mk<D4>(md.S0); in.S0.d[0] = 1.0;
    in.u = mk<D4>(md.u); in.u.d[1] = md.u * md.sq;
    D4 r = mk<D4>(md.r); r.d[2] = md.r * md.dt;
    in.d = mk<D4>(1.0) / in.u;
    in.rho = mk<D4>(1.0) / r;
    in.k = mk<D4>(md.k); in.k.d[3] = 1.0;
    in.K = mk<D4>(md.K);
    in.K2 = mk<D4>(md.K2);
    return in;
}

// Stage capacities of one node update (points).  W = max of the children,
// A and B the two halves of ENV, V the restricted function, Z the result.
struct Caps {
    int cW, cA, cB, cV, cZ;
    int64_t oW, oA, oB, oV, oZ, total;  // offsets / size in stride units
};

BTHD Caps make_caps(int cW, int cA, int cB, int cV, int cZ)
{
    Caps c;
    c.cW = cW; c.cA = cA; c.cB = cB; c.cV = cV; c.cZ = cZ;
    c.oW = 0;
    c.oA = c.oW + 3 * (int64_t)cW + 1;
    c.oB = c.oA + 3 * (int64_t)cA + 1;
    c.oV = c.oB + 3 * (int64_t)cB + 1;
    c.oZ = c.oV + 3 * (int64_t)cV + 1;
    c.total = c.oZ + 3 * (int64_t)cZ + 1;
    return c;
}

// Interleaved fast-path capacities (every stage SMALL_CAP points).
BTHD Caps small_caps() { return make_caps(SMALL_CAP, SMALL_CAP, SMALL_CAP, SMALL_CAP, SMALL_CAP); }

template <typename T>
BTD Arr<T> stage(T *base, int st, int64_t off, int cap)
{
    Arr<T> a;
    a.x = base + off * st;
    a.v = base + (off + cap) * st;
    a.s = base + (off + 2 * (int64_t)cap) * st;
    a.st = st;
    a.cap = cap;
    return a;
}

template <typename T>
BTD T pos_part(const T &x)
{
    return val(x) > 0.0 ? x : mk<T>(0.0);
}

// Exercise payoff (xi, zeta) at stock price S (Section 3: xi in cash and
// zeta shares; settled by delivery or in cash).  Delivered: put (K, -1),
// call (-K, 1).  In cash (zeta = 0): bull spread (S-K)^+ - (S-K2)^+
// (Section 5), put (K-S)^+, call (S-K)^+, bear spread (K2-S)^+ - (K-S)^+,
// straddle |S-K|.
template <typename T>
BTD void payoff(const Model &md, const Inputs<T> &in, const T &S, T &xi, T &zeta)
{
    zeta = mk<T>(0.0);
    switch (md.payoff) {
    case PAY_PUT: xi = in.K; zeta = mk<T>(-1.0); break;
    case PAY_CALL: xi = -in.K; zeta = mk<T>(1.0); break;
    case PAY_BULL: xi = pos_part(S - in.K) - pos_part(S - in.K2); break;
    case PAY_PUT_CASH: xi = pos_part(in.K - S); break;
    case PAY_CALL_CASH: xi = pos_part(S - in.K); break;
    case PAY_BEAR: xi = pos_part(in.K2 - S) - pos_part(in.K - S); break;
    default: {
        const T e = S - in.K;
        xi = val(e) > 0.0 ? e : -e;
    }
    }
}

// base^n by binary powering, multiplying in base^(2^i) for each set bit i
// in increasing i (the stock lattice S0 u^j of Section 4.1).
template <typename T>
BTD T upow(const T &base, int n)
{
    T acc = mk<T>(1.0), b = base;
    bool first = true;
    while (n > 0) {
        if (n & 1) { acc = first ? b : acc * b; first = false; }
        n >>= 1;
        if (n) b = b * b;
    }
    return acc;
}

// Stock price at lattice index j: S0 u^j (j >= 0) or S0 d^-j.
template <typename T>
BTD T stock_at(const Inputs<T> &in, int j)
{
    return in.S0 * (j >= 0 ? upow(in.u, j) : upow(in.d, -j));
}

// The optimal stock holding at t = 0, the hedge (Section 3: the root's
// restriction is the cheapest way to rebalance from no shares): with
// f = rho max(Zu, Zd) and g(y) = f(y) + Sa y for y >= 0, f(y) + Sb y for
// y < 0 (Sa, Sb the stock's ask and bid prices at t = 0), the minimum of g is
// at f's breakpoints or at 0; [lo, hi] is the range of those candidates
// whose g is within 1e-12 (relative, floor 1) of the smallest.  buf holds
// 3 cap + 1 numbers.  false when f has more than cap points.
template <typename T>
BTD bool root_hedge(const View<T> &Zu, const View<T> &Zd, const T &rho, double Sa, double Sb, T *buf, int cap,
                    double *lo, double *hi)
{
    Arr<T> W;
    W.x = buf;
    W.v = buf + cap;
    W.s = buf + 2 * (int64_t)cap;
    W.st = 1;
    W.cap = cap;
    int m = merge<OPMAX, T>(Zu, Zd, W);
    if (m < 0) return false;
    m = scale(W, m, rho);
    const View<T> f = W.view(m);
    double gmin = __builtin_huge_val();
    for (int pass = 0; pass < 2; pass++) {
        bool first = true;
        for (int j = 0; j <= m; j++) {
            const double y = j < m ? val(f.X(j)) : 0.0;
            const double g = val(eval(f, mk<T>(y))) + (y >= 0.0 ? Sa * y : Sb * y);
            if (pass == 0) {
                gmin = g < gmin ? g : gmin;
            } else if (g <= gmin + 1e-12 * fmax(1.0, fabs(gmin))) {
                if (first || y < *lo) *lo = y;
                if (first || y > *hi) *hi = y;
                first = false;
            }
        }
    }
    return true;
}

// Whether exercise attains the party's expense at zero stock holding
// (Section 3): the seller's z_t is max(u_t, v_t), so 1 when u_t(0) >=
// v_t(0); the buyer's is min(u_t, v_t), so 1 when u_t(0) <= v_t(0).  u_t is
// the kink at zeta (seller) or -zeta (buyer) with value xi or -xi and slopes
// a, b; both values are taken by EVAL.
template <int SIDE, typename T>
BTD int exercise_flag(const View<T> &V, const T &xi, const T &zeta, const T &a, const T &b)
{
    const T x0 = SIDE == 0 ? zeta : -zeta;
    const T u0 = SIDE == 0 ? xi : -xi;
    const T y = mk<T>(0.0);
    const double u = val(u0 + (val(x0) <= 0.0 ? b : a) * (y - x0));
    const double v = val(eval(V, y));
    return SIDE == 0 ? (u >= v ? 1 : 0) : (u <= v ? 1 : 0);
}

// One node of the seller's (SIDE 0) or buyer's (SIDE 1) recursion,
// Section 3: W = max(z_up, z_down); F = rho W; V = F with slopes restricted
// to [a, b] = [-(1+k_t) S, -(1-k_t) S] (CLIP for the convex seller, ENV for
// the buyer); U = the expense function u_t (kink at zeta, value xi for the
// seller; kink at -zeta, value -xi for the buyer); Z = max(U, V) for the
// seller, min(U, V) for the buyer, or Z = V when exercise is not allowed at
// t (European variant).  Temporaries live in `base` with element stride
// `st` and the capacities of `cp`.  Returns the point count of Z (whose
// storage is set in *zout) or -1 when a capacity was exceeded.  exf
// (binary64 only, optional) receives exercise_flag, 0 where exercise is not
// allowed.
template <int SIDE, typename T>
BTD int node_update(const View<T> &Zu, const View<T> &Zd, const T &S, const T &kt, const T &rho,
                    const T &xi, const T &zeta, bool exercise, T *base, int st,
                    const Caps &cp, Arr<T> *zout, int *exf = nullptr)
{
    const T one = mk<T>(1.0);
    const T a = -((one + kt) * S);
    const T b = -((one - kt) * S);
    Arr<T> W = stage(base, st, cp.oW, cp.cW);
    const int mw = merge_scale<OPMAX, T>(Zu, Zd, W, rho);
    if (mw < 0) return -1;
    Arr<T> V;
    int mv;
    if (SIDE == 0) {
        mv = clip(W, mw, a, b);
        V = W;
    } else {
        V = stage(base, st, cp.oV, cp.cV);
        const View<T> Fv = W.view(mw);
        if (val(a) == val(b)) {
            int js = 0;
            double best = 0.0;
            for (int j = 0; j < mw; j++) {
                const double h = val(Fv.V(j) - a * Fv.X(j));
                if (j == 0 || h < best) { best = h; js = j; }
            }
            const T xs = Fv.X(js), vs = Fv.V(js);
            V.X(0) = xs; V.V(0) = vs; V.S(0) = a; V.S(1) = a;
            mv = 1;
        } else {
            // the raw sweeps go to the A and B stages; A with its CANON lands
            // in the Z stage (free until the final MERGE), B = mirror(RB)
            // with its CANON in W (free once both sweeps have read F)
            Arr<T> A = stage(base, st, cp.oA, cp.cA);
            Arr<T> B = stage(base, st, cp.oB, cp.cB);
            Arr<T> Ac = stage(base, st, cp.oZ, cp.cZ);
            const int ma = sweep_a<false, T>(Fv, a, A, Ac);
            if (ma < 0) return -1;
            const int mr = sweep_raw<true, T>(Fv, -b, B);
            if (mr < 0) return -1;
            const int mb = mirror_canon_raw(B, mr, -b, W);
            if (mb < 0) return -1;
            mv = merge<OPMIN, T>(Ac.view(ma), W.view(mb), V);
            if (mv < 0) return -1;
        }
    }
    if constexpr (sizeof(T) == sizeof(double)) {
        if (exf) *exf = exercise ? exercise_flag<SIDE, T>(V.view(mv), xi, zeta, a, b) : 0;
    }
    if (!exercise) { *zout = V; return mv; }
    const Kink<T> U{SIDE == 0 ? zeta : -zeta, SIDE == 0 ? xi : -xi, a, b, 1};
    Arr<T> Z = stage(base, st, cp.oZ, cp.cZ);
    const int mz = merge<SIDE == 0 ? OPMAX : OPMIN, T>(U, V.view(mv), Z);
    *zout = Z;
    return mz;
}

}  // namespace bt
