// bt_cpu_alg1.cpp -- the paper's block/region partition (Section 4.2,
// Algorithm 1) on host threads: the CPU baseline of libbtcpu (bt_cpu.h).
//
// Built with the host compiler and BT_HOST_BUILD, so that the per-node
// update of Section 3 is the very code the GPU kernels run (bt_device.hpp):
// results are the same bits.
#define BT_HOST_BUILD 1
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/bt_cpu.h"
#include "bt_device.hpp"

using namespace bt;

namespace {

constexpr int MAX_THREADS = 64;

// One expense function: [s_0, (x_j, v_j, s_j+1)...] as in the GPU records.
struct Rec {
    std::vector<double> d;
    int m = 0;
    View<double> view() const { return View<double>{d.data() + 1, d.data() + 2, d.data(), m, 3}; }
};

// Waits with a short spin before yielding: the threads own a core each, as
// in the paper's implementation, and a round's work is a few hundred
// microseconds, so a sleeping wait would cost more than the work.
template <class F>
void spin_until(F done)
{
    for (int k = 0; !done(); k++) {
        if (k > 4096) std::this_thread::yield();
    }
}

// A reusable barrier for a changing number of participants: every round the
// participants agree on its size (they all compute the same p).
class Barrier {
public:
    void wait(int count)
    {
        const int gen = gen_.load(std::memory_order_acquire);
        if (arrived_.fetch_add(1, std::memory_order_acq_rel) + 1 == count) {
            arrived_.store(0, std::memory_order_relaxed);
            gen_.store(gen + 1, std::memory_order_release);
        } else {
            spin_until([&] { return gen_.load(std::memory_order_acquire) != gen; });
        }
    }

private:
    std::atomic<int> arrived_{0};
    std::atomic<int> gen_{0};
};

// Signal G_i of Algorithm 1: set by thread i, awaited and cleared by i-1.
struct Signal {
    std::atomic<int> on{0};
    void set() { on.store(1, std::memory_order_release); }
    void wait_and_clear()
    {
        spin_until([&] { return on.load(std::memory_order_acquire) != 0; });
        on.store(0, std::memory_order_relaxed);
    }
};

// What one thread accumulates (kept on its own cache lines).
struct alignas(128) Tally {
    int64_t nodes = 0;
    int64_t bp_sum[2] = {0, 0};
    int bp_max[2] = {0, 0};
};

struct Shared {
    Model md;
    int N, L;
    std::vector<double> Stab;          // S0 u^j, j = -(N+1)..N+1
    std::vector<Rec> buf[2];           // (L+1) rows x (N+2) columns, seller / buyer
    Signal G[MAX_THREADS];
    Barrier bar;
    std::atomic<int> failed{0};
    Tally tally[MAX_THREADS];
    int rounds = 0;
    Rec &cell(int side, int t, int c) { return buf[side][(size_t)(t % (L + 1)) * (N + 2) + c]; }
};

// Threads working in a round whose base level B holds B+1 nodes: p drops
// until each has at least two.
int active_threads(int B, int p)
{
    while (B + 1 < 2 * p && p > 1) p--;
    return p;
}

// Columns [s, e) of thread i at base level B with p threads.
void columns(int B, int p, int i, int &s, int &e)
{
    const int w = (B + 1) / p;
    s = i * w;
    e = (i == p - 1) ? B + 1 : (i + 1) * w;
}

// Node (t, c) of both parties from level t+1.
bool compute_node(Shared &X, int t, int c, Tally &tl, std::vector<double> &tmp)
{
    const Model &md = X.md;
    const int N = X.N;
    const Inputs<double> in = inputs_of(md, 0.0);
    const double kt = (t >= 1 || (md.flags & F_COST_AT_T0)) ? md.k : 0.0;
    const bool ex = !((md.flags & F_EUROPEAN) && t < N);
    const double S = X.Stab[2 * c - t + N + 1];
    double xi, ze;
    payoff(md, in, S, xi, ze);
    for (int side = 0; side < 2; side++) {
        const Rec &d = X.cell(side, t + 1, c), &u = X.cell(side, t + 1, c + 1);
        const int cap = 4 * (d.m + u.m) + 16;
        const Caps cp = make_caps(cap, cap, cap, cap, cap);
        if ((int64_t)tmp.size() < cp.total) tmp.resize(cp.total);
        Arr<double> Z;
        const int m = side == 0 ? node_update<0, double>(u.view(), d.view(), S, kt, md.rho, xi, ze, ex, tmp.data(), 1, cp, &Z)
                                : node_update<1, double>(u.view(), d.view(), S, kt, md.rho, xi, ze, ex, tmp.data(), 1, cp, &Z);
        if (m < 0) return false;
        Rec &z = X.cell(side, t, c);
        z.d.resize(3 * (size_t)m + 1);
        z.d[0] = Z.S(0);
        for (int j = 0; j < m; j++) {
            z.d[1 + 3 * j] = Z.X(j);
            z.d[2 + 3 * j] = Z.V(j);
            z.d[3 + 3 * j] = Z.S(j + 1);
        }
        z.m = m;
        const int bp = (m == 1 && Z.S(0) == Z.S(1)) ? 0 : m;
        tl.bp_sum[side] += bp;
        tl.bp_max[side] = std::max(tl.bp_max[side], bp);
    }
    tl.nodes++;
    return true;
}

// Algorithm 1, executed by thread i of p0 threads.
void thread_main(Shared &X, int i, int p0)
{
    const int N = X.N, L = X.L;
    std::vector<double> tmp;
    Tally tl;
    struct Keep {
        Shared &X;
        Tally &tl;
        int i;
        ~Keep() { X.tally[i] = tl; }
    } keep{X, tl, i};
    int p = active_threads(N + 1, p0);
    if (i >= p) return;
    int B = N + 1, s, e;
    columns(B, p, i, s, e);
    // the leaves: payoff (0, 0) at time N+1, the liquidation function
    for (int c = s; c < e; c++) {
        const double S = X.Stab[2 * c];
        for (int side = 0; side < 2; side++) {
            Rec &z = X.cell(side, N + 1, c);
            z.d = {-((1.0 + X.md.k) * S), 0.0, 0.0, -((1.0 - X.md.k) * S)};
            z.m = 1;
        }
        tl.nodes++;
    }
    X.bar.wait(p);
    while (B > 0) {
        const int D = std::min(L, (B + 1) / p - 1);
        const int T = D > 1 ? B - D + 1 : B - D;   // level whose leftmost node sends G_i
        // region A: level C, columns [s, min(e - o, C + 1))
        int o = 1;
        for (int C = B - 1; C >= B - D; C--, o++) {
            const int m = std::min(e - o, C + 1);
            for (int l = s; l < m; l++) {
                if (!X.failed.load(std::memory_order_relaxed) && !compute_node(X, C, l, tl, tmp)) X.failed = 1;
                if (i > 0 && C == T && l == s) X.G[i].set();
            }
        }
        // region B: after the right neighbour's signal, the triangle of
        // columns [e - o, e) at level B - o
        if (i + 1 < p) {
            X.G[i + 1].wait_and_clear();
            for (int oo = 1; oo <= D; oo++) {
                const int C = B - oo;
                for (int l = e - oo; l < e; l++)
                    if (!X.failed.load(std::memory_order_relaxed) && !compute_node(X, C, l, tl, tmp)) X.failed = 1;
            }
        }
        X.bar.wait(p);
        B -= D;
        if (i == 0) X.rounds++;
        if (B > 0) {
            p = active_threads(B, p);
            if (i >= p) return;
            columns(B, p, i, s, e);
        }
    }
}

}  // namespace

extern "C" int bt_cpu_price(const bt_params *prm, int32_t threads, int32_t L, bt_result *out, bt_cpu_stats *stats)
{
    if (!prm || !out || threads < 1 || threads > MAX_THREADS || L < 1) return BT_EINVAL;
    const double nan = __builtin_nan("");
    bt_result r;
    r.ask = r.bid = r.price0 = nan;
    r.bp_total_ask = r.bp_total_bid = 0;
    r.bp_max_ask = r.bp_max_bid = 0;
    r.reserved = 0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Shared *X = new (std::nothrow) Shared();
    if (!X) return BT_ENOMEM;
    if (!derive_model(*prm, BT_MAX_N, X->md)) {
        delete X;
        r.status = BT_EINVAL;
        *out = r;
        return BT_OK;
    }
    const Model &md = X->md;
    const int N = md.N;
    X->N = N;
    X->L = L;
    const Inputs<double> in = inputs_of(md, 0.0);
    X->Stab.resize(2 * (size_t)N + 3);
    for (int idx = 0; idx < 2 * N + 3; idx++) X->Stab[idx] = stock_at(in, idx - (N + 1));
    for (int side = 0; side < 2; side++) X->buf[side].resize((size_t)(L + 1) * (N + 2));
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> pool;
    for (int i = 1; i < threads; i++) pool.emplace_back(thread_main, std::ref(*X), i, (int)threads);
    thread_main(*X, 0, threads);
    for (std::thread &t : pool) t.join();
    const auto t1 = std::chrono::steady_clock::now();
    if (X->failed) {
        r.status = BT_ENOMEM;
    } else {
        r.status = BT_OK;
        const View<double> za = X->cell(0, 0, 0).view(), zb = X->cell(1, 0, 0).view();
        r.ask = eval(za, 0.0);
        r.bid = -eval(zb, 0.0);
        for (int i = 0; i < threads; i++) {
            r.bp_total_ask += X->tally[i].bp_sum[0];
            r.bp_total_bid += X->tally[i].bp_sum[1];
            r.bp_max_ask = std::max(r.bp_max_ask, X->tally[i].bp_max[0]);
            r.bp_max_bid = std::max(r.bp_max_bid, X->tally[i].bp_max[1]);
        }
        // zero-cost price: the scalar recursion (Section 3, Appendix)
        std::vector<double> V(N + 1);
        const bool euro = (md.flags & F_EUROPEAN) != 0;
        for (int c = 0; c <= N; c++) {
            double xi, ze;
            const double S = X->Stab[2 * c + 1];
            payoff(md, in, S, xi, ze);
            const double P = xi + ze * S;
            V[c] = P > 0.0 ? P : 0.0;
        }
        const double pu = md.p, q = 1.0 - md.p, rho = md.rho;
        for (int t = N - 1; t >= 0; t--)
            for (int c = 0; c <= t; c++) {
                const double cont = rho * (pu * V[c + 1] + q * V[c]);
                if (euro) { V[c] = cont; continue; }
                double xi, ze;
                const double S = X->Stab[2 * c - t + N + 1];
                payoff(md, in, S, xi, ze);
                double P = xi + ze * S;
                if (P < 0.0) P = 0.0;
                V[c] = P > cont ? P : cont;
            }
        r.price0 = V[0];
    }
    if (stats) {
        stats->seconds = std::chrono::duration<double>(t1 - t0).count();
        for (int i = 0; i < threads; i++) stats->nodes[i] = X->tally[i].nodes;
        stats->threads = threads;
        stats->rounds = X->rounds;
    }
    *out = r;
    delete X;
    return BT_OK;
}
