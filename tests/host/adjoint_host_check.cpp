// The reverse sweep of the Greeks (bt_adjoint.hpp) built for the CPU and run
// on whole trees, one node at a time, with the checkpoint schedule of the
// GPU kernel: the forward pass keeps the levels t = N+1, N+1-s, ... (s =
// ceil(sqrt(N+2))); the reverse pass recomputes the levels between two
// checkpoints from the upper one, root side first, and steps back through
// them.  Used by the CPU tests to compare the adjoint with the oracle's
// tangents without a GPU.
//
// stdin, one option per line: S0 K K2 R sigma T k N payoff flags
// stdout, one line per option: error ask bid total_bp_ask total_bp_bid
// max_bp_ask max_bp_bid [8 derivatives: ask then bid by S0, sigma, R, k]
// peak_tape peak_points, numbers in hexadecimal floating point.
#define BT_HOST_DEBUG 1
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>
#include "bt_adjoint.hpp"
using namespace bt;

struct Level {
    std::vector<double> rec;
    std::vector<int> off, cnt;   // per column
};

static View<double> rview(const Level &L, int c)
{
    const double *r = L.rec.data() + L.off[c];
    return View<double>{r + 1, r + 2, r, L.cnt[c], 3};
}

static long long g_peak_tape = 0, g_peak_pts = 0;

// Level t from level t+1 (t+1 columns), per-lane path with room for any size.
template <int SIDE>
static int step_forward(const Model &md, const std::vector<double> &Stab, const Level &up, int t, Level &out,
                        long long *bp_tot, int *bp_max)
{
    const int N = md.N;
    const double k = md.k;
    const double kt = (t >= 1 || (md.flags & F_COST_AT_T0)) ? k : 0.0;
    const bool ex = !((md.flags & F_EUROPEAN) && t < N);
    const Inputs<double> in = inputs_of(md, 0.0);
    out.rec.clear();
    out.off.assign(t + 1, 0);
    out.cnt.assign(t + 1, 0);
    for (int c = 0; c <= t; c++) {
        const View<double> Zd = rview(up, c), Zu = rview(up, c + 1);
        const int M = Zd.m + Zu.m;
        const int cap = 4 * M + 16;
        const Caps cp = make_caps(cap, cap, cap, cap, cap);
        std::vector<double> tmp(cp.total + 8);
        const double S = Stab[2 * c - t + N + 1];
        double xi, ze;
        payoff(md, in, S, xi, ze);
        Arr<double> Z;
        const int m = node_update<SIDE, double>(Zu, Zd, S, kt, md.rho, xi, ze, ex, tmp.data(), 1, cp, &Z);
        if (m < 0) return -1;
        out.off[c] = (int)out.rec.size();
        out.cnt[c] = m;
        out.rec.push_back(Z.S(0));
        for (int j = 0; j < m; j++) {
            out.rec.push_back(Z.X(j));
            out.rec.push_back(Z.V(j));
            out.rec.push_back(Z.S(j + 1));
        }
        const int bp = (m == 1 && Z.S(0) == Z.S(1)) ? 0 : m;
        *bp_tot += bp;
        *bp_max = std::max(*bp_max, bp);
    }
    return 0;
}

template <int SIDE>
static int run_side(const Model &md, double *price, double *grad, long long *tot, int *mx)
{
    const int N = md.N;
    std::vector<double> Stab(2 * N + 3), Sfac(2 * N + 3);
    const Inputs<double> in = inputs_of(md, 0.0);
    for (int idx = 0; idx < 2 * N + 3; idx++) {
        const int j = idx - (N + 1);
        Sfac[idx] = j >= 0 ? upow(md.u, j) : upow(md.d, -j);
        Stab[idx] = stock_at(in, j);
    }
    int s = 1;
    while ((long long)s * s < N + 2) s++;
    // forward: leaves, then levels N..1; checkpoints at N+1, N+1-s, ...
    std::map<int, Level> cps;
    Level cur;
    cur.off.resize(N + 2);
    cur.cnt.assign(N + 2, 1);
    for (int c = 0; c <= N + 1; c++) {
        const double S = Stab[2 * c];
        cur.off[c] = 4 * c;
        cur.rec.insert(cur.rec.end(), {-(1.0 + md.k) * S, 0.0, 0.0, -(1.0 - md.k) * S});
    }
    cps[N + 1] = cur;
    *tot = 0;
    *mx = 0;
    for (int t = N; t >= 1; t--) {
        Level nx;
        if (step_forward<SIDE>(md, Stab, cur, t, nx, tot, mx)) return -1;
        cur.rec.swap(nx.rec); cur.off.swap(nx.off); cur.cnt.swap(nx.cnt);
        if ((N + 1 - t) % s == 0) cps[t] = cur;
    }
    // reverse: segments between checkpoints, root side first
    std::vector<int> cpl;
    for (auto &kv : cps) cpl.push_back(kv.first);   // ascending
    double gS0 = 0, gsig = 0, gR = 0, gk = 0;
    std::vector<double> Acur, Anxt;
    const bool t0cost = (md.flags & F_COST_AT_T0) != 0;
    int lo = 0;
    for (size_t ci = 0; ci < cpl.size(); ci++) {
        const int hi = cpl[ci];
        // levels lo+1 .. hi: hi from the checkpoint, the rest recomputed
        std::map<int, Level> seg;
        seg[hi] = cps[hi];
        for (int t = hi - 1; t >= lo + 1; t--) {
            long long dt_ = 0;
            int dm_ = 0;
            if (step_forward<SIDE>(md, Stab, seg[t + 1], t, seg[t], &dt_, &dm_)) return -1;
        }
        if (lo >= 1) seg[lo] = cps[lo];
        for (int t = lo; t <= hi - 1; t++) {
            const Level &Lc = seg[t + 1];
            Anxt.assign(Lc.rec.size(), 0.0);
            const double kt = (t >= 1 || t0cost) ? md.k : 0.0;
            const bool ex = !((md.flags & F_EUROPEAN) && t < N);
            for (int par = 0; par < 2; par++)
                for (int c = par; c <= t; c += 2) {
                    const View<double> Zd = rview(Lc, c), Zu = rview(Lc, c + 1);
                    const int M = Zd.m + Zu.m;
                    const int cap = 4 * M + 16;
                    const int tcap = 200 * M + 2000;
                    const RevCaps rc = rev_caps(cap, std::max(Zd.m, Zu.m), tcap);
                    std::vector<TN> tn(rc.tn);
                    std::vector<TapeEnt> ent(tcap);
                    std::vector<double> adj(3 * M + 5 + tcap);
                    std::vector<double> gd(3 * Zd.m + 1), gu(3 * Zu.m + 1);
                    const double S = Stab[2 * c - t + N + 1];
                    double g[3], pr = 0.0;
                    const double *zbar = nullptr;
                    int mz = 0;
                    if (t >= 1) {
                        const Level &Lt = seg[t];
                        zbar = Acur.data() + Lt.off[c];
                        mz = Lt.cnt[c];
                    }
                    if (node_reverse<SIDE>(md, Zd, Zu, S, kt, md.rho, ex, zbar, mz, rc, tn.data(), 0, ent.data(),
                                           adj.data(), gd.data(), gu.data(), g, &pr))
                        return -2;
                    g_peak_tape = std::max<long long>(g_peak_tape, bt_tape[0].n);
                    g_peak_pts = std::max<long long>(g_peak_pts, M);
                    if (t == 0) {
                        *price = SIDE == 0 ? pr : -pr;
                        // counts of level 0
                        long long d0 = 0;
                        int m0 = 0;
                        Level L0;
                        step_forward<SIDE>(md, Stab, Lc, 0, L0, &d0, &m0);
                        *tot += d0;
                        *mx = std::max(*mx, m0);
                    }
                    for (int q = 0; q < 3 * Zd.m + 1; q++) Anxt[Lc.off[c] + q] += gd[q];
                    for (int q = 0; q < 3 * Zu.m + 1; q++) Anxt[Lc.off[c + 1] + q] += gu[q];
                    const int j = 2 * c - t;
                    gS0 += g[0] * Sfac[j + N + 1];
                    gsig += g[0] * (S * (double)j * md.sq);
                    gR += g[2] * (-md.dt * md.rho);
                    if (t >= 1 || t0cost) gk += g[1];
                }
            Acur.swap(Anxt);
        }
        lo = hi;
    }
    // level N+1: [-(1+k) S, 0, 0, -(1-k) S] per column
    for (int c = 0; c <= N + 1; c++) {
        const double S = Stab[2 * c];
        const double a0 = Acur[4 * c], a1 = Acur[4 * c + 3];
        const double gSl = -(1.0 + md.k) * a0 - (1.0 - md.k) * a1;
        const int j = 2 * c - (N + 1);
        gS0 += gSl * Sfac[j + N + 1];
        gsig += gSl * (S * (double)j * md.sq);
        gk += -S * a0 + S * a1;
    }
    grad[0] = gS0; grad[1] = gsig; grad[2] = gR; grad[3] = gk;
    return 0;
}

int main()
{
    double S0, K, K2, R, sig, T, k;
    int N, pay;
    unsigned fl;
    while (scanf("%lf %lf %lf %lf %lf %lf %lf %d %d %u", &S0, &K, &K2, &R, &sig, &T, &k, &N, &pay, &fl) == 10) {
        bt_params p{S0, K, K2, R, sig, T, k, N, pay, fl, 0u};
        Model m{};
        if (!derive_model(p, BT_MAX_N, m)) { printf("-1\n"); fflush(stdout); continue; }
        double pa = 0, pb = 0, ga[4], gb[4];
        long long ta = 0, tb = 0;
        int ma = 0, mb = 0;
        const int e1 = run_side<0>(m, &pa, ga, &ta, &ma), e2 = run_side<1>(m, &pb, gb, &tb, &mb);
        printf("%d %a %a %lld %lld %d %d %a %a %a %a %a %a %a %a %lld %lld\n", e1 | e2, pa, pb, ta, tb, ma, mb, ga[0],
               ga[1], ga[2], ga[3], gb[0], gb[1], gb[2], gb[3], g_peak_tape, g_peak_pts);
        fflush(stdout);
    }
}
