// bt_adjoint.hpp -- reverse-mode derivatives of the ask and bid: numbers
// that record their arithmetic on a tape, and the reverse step of one node.
//
// The reverse sweep runs the recursion of Section 3 backwards.  Level t's
// adjoint holds, for every number of every record of level t (the expense
// functions z_t(c) stored as [s_0, (x_j, v_j, s_j+1)...]), the derivative of
// the price with respect to that number.  The reverse step of node (t, c)
// recomputes z_t(c) from its two children with numbers of type TN, each of
// which records the operation that made it; then the tape is read backwards
// from the adjoint of z_t(c) (at the root: the derivative of the price
// z_0(0), +1 for the seller's ask, -1 for the buyer's bid), which gives the
// adjoints of the children's numbers and of the node's own inputs: its stock
// price S, cost rate k_t and discount rho.  Those three turn into the Greeks
// through dS/dS0 = S/S0, dS/dsigma = S (2c - t) sqrt(T/N), drho/dR = -rho T/N
// and dk_t/dk = 1.  The recomputation takes the same operations in the same
// order as the forward pass, so it reproduces the stored record bit for bit.
#pragma once

#include "bt_device.hpp"

namespace bt {

// One lane's tape.  Entry e records r = f(a, b) as (id of a, id of b,
// dr/da, dr/db); r gets the id base + e.  Ids below base name the node's
// inputs (its children's record numbers, then S, k_t, rho); -1 is a
// constant.  ovf is set when an entry did not fit (the step then fails).
// The entries live in global memory; each lane's header (count, capacity,
// base, entries) lives in LDS on the GPU, so that recording an operation
// costs no round trip to memory for the count.
struct TapeEnt {
    int32_t ia, ib;
    double pa, pb;
};

struct TapeHdr {
    int32_t n, cap, base, ovf;
    TapeEnt *ent;
};

constexpr int TAPE_SLOTS = 256;   // one per lane of a workgroup
#ifdef BT_HOST_DEBUG
inline TapeHdr bt_tape[TAPE_SLOTS];
#else
__shared__ TapeHdr bt_tape[TAPE_SLOTS];
#endif

// A number that records the operations that made it on the tape of slot
// `lane` (-1: a constant).
struct TN {
    double v;
    int32_t id;
    int32_t lane;
};

BTD double val(const TN &x) { return x.v; }
template <> BTD TN mk<TN>(double x)
{
    TN r;
    r.v = x;
    r.id = -1;
    r.lane = -1;
    return r;
}

BTD TN tn_rec(double v, const TN &a, double pa, const TN &b, double pb)
{
    TN r;
    r.v = v;
    r.id = -1;
    r.lane = a.lane >= 0 ? a.lane : b.lane;
    if (r.lane < 0 || (a.id < 0 && b.id < 0)) return r;
    TapeHdr &t = bt_tape[r.lane];
    const int e = t.n;
    if (e >= t.cap) {
        t.ovf = 1;
        return r;
    }
    t.n = e + 1;
    TapeEnt q;
    q.ia = a.id;
    q.ib = b.id;
    q.pa = pa;
    q.pb = pb;
    t.ent[e] = q;
    r.id = t.base + e;
    return r;
}

BTD TN operator+(const TN &a, const TN &b) { return tn_rec(a.v + b.v, a, 1.0, b, 1.0); }
BTD TN operator-(const TN &a, const TN &b) { return tn_rec(a.v - b.v, a, 1.0, b, -1.0); }
BTD TN operator*(const TN &a, const TN &b) { return tn_rec(a.v * b.v, a, b.v, b, a.v); }
BTD TN operator/(const TN &a, const TN &b)
{
    const double q = a.v / b.v;
    return tn_rec(q, a, 1.0 / b.v, b, -q / b.v);
}
BTD TN operator-(const TN &a) { return tn_rec(-a.v, a, -1.0, mk<TN>(0.0), 0.0); }

// Numbers one reverse step needs for a node whose children hold mu + md
// points and whose stages hold at most `cap` points each.
struct RevCaps {
    Caps cp;            // stage capacities (TN numbers, element stride 1)
    int64_t tn;         // TN numbers: stages + the two child copies
    int32_t tape;       // tape entries
};

BTHD RevCaps rev_caps(int cap, int child_cap, int tape)
{
    RevCaps r;
    r.cp = make_caps(cap, cap, cap, cap, cap);
    r.tn = r.cp.total + 2 * (3 * (int64_t)child_cap + 1);
    r.tape = tape;
    return r;
}

// Reverse step of node (t, c) of the seller (SIDE 0) or the buyer (SIDE 1).
//   Zd, Zu   the children's records (z_t+1(c), z_t+1(c+1)), values only;
//   S, kt, rho, exercise as in node_update;
//   zbar     the adjoint of z_t(c)'s record numbers in record order, or
//            nullptr at the root (seed d price / d z_0(0));
//   mz       the point count of z_t(c) in the forward pass (nullptr zbar:
//            ignored);
//   tn       TN scratch of rc.tn numbers; ent room for rc.tape tape
//            entries, recorded through tape slot `slot`;
//   adj      scratch of 3 (mu + md) + 5 + rc.tape doubles;
//   gd, gu   out: the adjoints of the children's record numbers
//            (3 md + 1 and 3 mu + 1 of them);
//   g        out: adjoints of S, k_t, rho; price: out, z_t(c) at y = 0 at
//            the root (the ask, or minus the bid).
// Returns 0, or -1 when the scratch or the tape was too small (or the
// recomputed record does not have mz points).
template <int SIDE>
BTD int node_reverse(const Model &md, const View<double> &Zd, const View<double> &Zu, double S, double kt,
                     double rho, bool exercise, const double *zbar, int mz, const RevCaps &rc, TN *tn, int slot,
                     TapeEnt *ent, double *adj, double *gd, double *gu, double *g, double *price)
{
    const int nd = 3 * Zd.m + 1, nu = 3 * Zu.m + 1;
    if (nd + nu > rc.tn - rc.cp.total) return -1;
    TN *cd = tn + rc.cp.total;
    TN *cu = cd + nd;
    // the children's numbers: record position k of z_t+1(c) has id k, of
    // z_t+1(c+1) id nd + k
    for (int k = 0; k < nd; k++) {
        const double x = k == 0 ? Zd.S(0) : ((k - 1) % 3 == 0 ? Zd.X((k - 1) / 3)
                                                             : ((k - 1) % 3 == 1 ? Zd.V((k - 1) / 3) : Zd.S((k - 1) / 3 + 1)));
        cd[k].v = x; cd[k].id = k; cd[k].lane = slot;
    }
    for (int k = 0; k < nu; k++) {
        const double x = k == 0 ? Zu.S(0) : ((k - 1) % 3 == 0 ? Zu.X((k - 1) / 3)
                                                             : ((k - 1) % 3 == 1 ? Zu.V((k - 1) / 3) : Zu.S((k - 1) / 3 + 1)));
        cu[k].v = x; cu[k].id = nd + k; cu[k].lane = slot;
    }
    const int pS = nd + nu, pK = pS + 1, pR = pS + 2;
    TapeHdr &tp = bt_tape[slot];
    tp.n = 0;
    tp.cap = rc.tape;
    tp.ovf = 0;
    tp.base = pS + 3;
    tp.ent = ent;
    TN tS = mk<TN>(S), tK = mk<TN>(kt), tR = mk<TN>(rho);
    tS.id = pS; tS.lane = slot;
    tK.id = pK; tK.lane = slot;
    tR.id = pR; tR.lane = slot;
    Inputs<TN> in;
    in.S0 = in.u = in.d = in.rho = in.k = mk<TN>(0.0);
    in.K = mk<TN>(md.K);
    in.K2 = mk<TN>(md.K2);
    TN xi, ze;
    payoff(md, in, tS, xi, ze);
    const View<TN> Vd{cd + 1, cd + 2, cd, Zd.m, 3}, Vu{cu + 1, cu + 2, cu, Zu.m, 3};
    Arr<TN> Z;
    const int m = node_update<SIDE, TN>(Vu, Vd, tS, tK, tR, xi, ze, exercise, tn, 1, rc.cp, &Z);
    if (m < 0 || tp.ovf) return -1;
    TN root = mk<TN>(0.0);
    if (!zbar) {
        root = eval(Z.view(m), mk<TN>(0.0));
        if (tp.ovf) return -1;
        *price = root.v;
    } else if (m != mz) {
        return -1;
    }
    const int total = tp.base + tp.n;
    for (int i = 0; i < total; i++) adj[i] = 0.0;
    if (!zbar) {
        if (root.id >= 0) adj[root.id] += SIDE == 0 ? 1.0 : -1.0;
    } else {
        if (Z.S(0).id >= 0) adj[Z.S(0).id] += zbar[0];
        for (int j = 0; j < m; j++) {
            if (Z.X(j).id >= 0) adj[Z.X(j).id] += zbar[1 + 3 * j];
            if (Z.V(j).id >= 0) adj[Z.V(j).id] += zbar[2 + 3 * j];
            if (Z.S(j + 1).id >= 0) adj[Z.S(j + 1).id] += zbar[3 + 3 * j];
        }
    }
    const int base = tp.base;
    for (int e = tp.n - 1; e >= 0; e--) {
        const double a = adj[base + e];
        if (a == 0.0) continue;
        const TapeEnt q = ent[e];
        if (q.ia >= 0) adj[q.ia] += a * q.pa;
        if (q.ib >= 0) adj[q.ib] += a * q.pb;
    }
    for (int k = 0; k < nd; k++) gd[k] = adj[k];
    for (int k = 0; k < nu; k++) gu[k] = adj[nd + k];
    g[0] = adj[pS];
    g[1] = adj[pK];
    g[2] = adj[pR];
    return 0;
}

}  // namespace bt
