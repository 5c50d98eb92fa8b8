// bt_kernels.hip -- gfx950 kernels of libbtprice and the C ABI around them.
//
// One persistent kernel prices a book.  Every option contributes three work
// items -- the seller's recursion (ask), the buyer's recursion (bid) and the
// zero-cost recursion (price0) -- handed out longest-first from a queue in
// device memory.  A workgroup of 256 lanes takes one item at a time and
// sweeps its tree from level N+1 to the root (Section 3 recursions; tree of
// Section 4.1), one lane per node and 256 nodes per chunk, holding the
// current and the next level as packed variable-length records.  Node
// temporaries live in an interleaved per-lane area (coalesced across the
// wave); a node whose breakpoints overflow it is redone on a pool path whose
// capacities cannot be exceeded, admitted by a workgroup prefix sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/bt.h"
#include "bt_device.hpp"

using namespace bt;

namespace {

struct KArgs {
    const Model *models;
    const int *sched;
    int n_items;
    int *queue;
    bt_result *out;
    double *ws;
    int64_t ws_doubles;  // per workgroup
    int *wsi;
    int64_t wsi_ints;    // per workgroup
    int n_max;
    int64_t lcapd;       // doubles per level buffer
    int64_t pool;        // doubles in the pool
    int64_t oStab, oL0, oL1, oSmall, oPool;
};

// Exclusive prefix sum over the workgroup; *total gets the sum.
__device__ __forceinline__ int64_t block_scan(int64_t v, int64_t *total, int64_t *sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; w++) {
        int64_t t = sh[w];
        base += (w < wid) ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__device__ __forceinline__ View record_view(const double *L, int64_t off, int m)
{
    return View{L + off + 1, L + off + 2, L + off, m, 3};
}

__device__ __forceinline__ void write_record(double *dst, const Arr &z, int m)
{
    dst[0] = z.S(0);
    for (int j = 0; j < m; j++) {
        dst[1 + 3 * j] = z.X(j);
        dst[2 + 3 * j] = z.V(j);
        dst[3 + 3 * j] = z.S(j + 1);
    }
}

__device__ void stock_table(const Model &md, double *Stab)
{
    const int N = md.N;
    for (int idx = threadIdx.x; idx < 2 * N + 3; idx += WG) {
        int j = idx - (N + 1);
        double f = j >= 0 ? upow(md.u, j) : upow(md.d, -j);
        Stab[idx] = md.S0 * f;
    }
}

// Zero-cost recursion (Section 3, Appendix): no extra level;
// V_N = max(xi + zeta S, 0), V_t = max(xi + zeta S, rho (p V_up + (1-p) V_dn))
// (European variant: V_t = continuation value).
__device__ void price0_item(const KArgs &A, const Model &md, int opt, double *ws)
{
    const int N = md.N;
    double *Stab = ws + A.oStab;
    double *V0 = ws + A.oL0, *V1 = ws + A.oL1;
    stock_table(md, Stab);
    __syncthreads();
    const bool euro = (md.flags & F_EUROPEAN) != 0;
    for (int c = threadIdx.x; c <= N; c += WG) {
        double S = Stab[2 * c + 1], xi, ze;
        payoff(md, S, xi, ze);
        double P = xi + ze * S;
        V0[c] = P > 0.0 ? P : 0.0;
    }
    __syncthreads();
    const double p = md.p, q = 1.0 - md.p, rho = md.rho;
    double *cur = V0, *nxt = V1;
    for (int t = N - 1; t >= 0; t--) {
        for (int c = threadIdx.x; c <= t; c += WG) {
            double cont = rho * (p * cur[c + 1] + q * cur[c]);
            if (euro) { nxt[c] = cont; continue; }
            double S = Stab[2 * c - t + N + 1], xi, ze;
            payoff(md, S, xi, ze);
            double P = xi + ze * S;
            if (P < 0.0) P = 0.0;
            nxt[c] = P > cont ? P : cont;
        }
        __syncthreads();
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (threadIdx.x == 0) A.out[opt].price0 = cur[0];
}

// Seller (SIDE 0) or buyer (SIDE 1) recursion of Section 3 for one option.
template <int SIDE>
__device__ void side_item(const KArgs &A, const Model &md, int opt, double *ws, int *wsi,
                          int64_t *sh, int *sflag)
{
    const int N = md.N;
    const int tid = threadIdx.x;
    double *Stab = ws + A.oStab;
    double *Lb[2] = {ws + A.oL0, ws + A.oL1};
    int *offb[2] = {wsi, wsi + 2 * (A.n_max + 2)};
    int *cntb[2] = {wsi + (A.n_max + 2), wsi + 3 * (A.n_max + 2)};
    double *small = ws + A.oSmall;
    double *pool = ws + A.oPool;

    stock_table(md, Stab);
    if (tid == 0) *sflag = 0;
    __syncthreads();
    // level N+1: liquidation y^- S^a - y^+ S^b (payoff (0, 0)), record
    // [s0, x0, v0, s1] = [-(1+k) S, 0, 0, -(1-k) S]
    for (int c = tid; c <= N + 1; c += WG) {
        double S = Stab[2 * c];
        double Sa = (1.0 + md.k) * S, Sb = (1.0 - md.k) * S;
        double *r = Lb[0] + 4 * (int64_t)c;
        r[0] = -Sa; r[1] = 0.0; r[2] = 0.0; r[3] = -Sb;
        offb[0][c] = 4 * c;
        cntb[0][c] = 1;
    }
    __syncthreads();

    const Caps sc = small_caps();
    const bool euro = (md.flags & F_EUROPEAN) != 0;
    int64_t bp_sum = 0;
    int bp_max = 0;
    bool fatal = false;
    int cur = 0;
    for (int t = N; t >= 0 && !fatal; t--) {
        const double kt = (t >= 1 || (md.flags & F_COST_AT_T0)) ? md.k : 0.0;
        const bool exercise = !(euro && t < N);
        const double *Lc = Lb[cur];
        const int *offc = offb[cur], *cntc = cntb[cur];
        double *Ln = Lb[cur ^ 1];
        int *offn = offb[cur ^ 1], *cntn = cntb[cur ^ 1];
        int64_t loff = 0;
        for (int cb = 0; cb <= t && !fatal; cb += WG) {
            const int c = cb + tid;
            const bool act = c <= t;
            View Zu{}, Zd{};
            double S = 0.0, xi = 0.0, ze = 0.0;
            int M = 0;
            if (act) {
                Zd = record_view(Lc, offc[c], cntc[c]);
                Zu = record_view(Lc, offc[c + 1], cntc[c + 1]);
                M = cntc[c] + cntc[c + 1];
                S = Stab[2 * c - t + N + 1];
                payoff(md, S, xi, ze);
            }
            // Rounds: round 0 runs every node on the interleaved area; later
            // rounds rerun the nodes that overflowed it on the pool, tier 1
            // with generous capacities, tier 2 with capacities that cannot be
            // exceeded, admitted by a prefix sum over the pool size.
            int tier = act ? 0 : -1;
            for (int round = 0; !fatal; round++) {
                if (round > 0 && !__syncthreads_or(tier >= 1)) break;
                Caps cp = sc;
                double *base = small + tid;
                int st = WG;
                bool run = (round == 0) ? (tier == 0) : false;
                if (round > 0) {
                    cp = tier == 2 ? big_caps(M, SIDE == 1) : pool_caps(M, SIDE == 1);
                    int64_t need = tier >= 1 ? cp.total : 0, ntot;
                    int64_t nex = block_scan(need, &ntot, sh);
                    run = tier >= 1 && (nex + need <= A.pool);
                    if (tier >= 1 && nex == 0 && need > A.pool) *sflag = 1;
                    base = pool + nex;
                    st = 1;
                }
                Arr Z{};
                int mz = 0;
                if (run) {
                    mz = node_update<SIDE>(Zu, Zd, S, kt, md.rho, xi, ze, exercise, base, st, cp, &Z);
                    if (mz < 0 && tier == 2) *sflag = 1;
                }
                int64_t sz = (run && mz > 0) ? 3 * (int64_t)mz + 1 : 0, tot;
                int64_t ex = block_scan(sz, &tot, sh);
                if (*sflag || loff + tot > A.lcapd) {
                    fatal = true;
                } else if (sz) {
                    write_record(Ln + loff + ex, Z, mz);
                    offn[c] = (int)(loff + ex);
                    cntn[c] = mz;
                    int bp = (mz == 1 && Z.S(0) == Z.S(1)) ? 0 : mz;
                    bp_sum += bp;
                    bp_max = bp > bp_max ? bp : bp_max;
                }
                loff += tot;
                if (run) tier = (mz > 0) ? -1 : (tier == 0 ? 1 : 2);
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    // workgroup reduction of the breakpoint statistics
    __shared__ int64_t rs[NWAVE];
    __shared__ int rm[NWAVE];
    int64_t s = bp_sum;
    int mx = bp_max;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_down(s, o, 64);
        int y = __shfl_down(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if ((tid & 63) == 0) { rs[tid >> 6] = s; rm[tid >> 6] = mx; }
    __syncthreads();
    if (tid == 0) {
        int64_t ts = 0;
        int tm = 0;
        for (int w = 0; w < NWAVE; w++) { ts += rs[w]; tm = rm[w] > tm ? rm[w] : tm; }
        bt_result &o = A.out[opt];
        if (fatal) {
            atomicMin(&o.status, BT_EOVERFLOW);
        } else {
            View z0 = record_view(Lb[cur], offb[cur][0], cntb[cur][0]);
            double root = eval(z0, 0.0);
            if (SIDE == 0) { o.ask = root; o.bp_total_ask = ts; o.bp_max_ask = tm; }
            else { o.bid = -root; o.bp_total_bid = ts; o.bp_max_bid = tm; }
        }
    }
    __syncthreads();
}

// One persistent kernel per kind of work item (ask, bid, price0), each with
// its own longest-first queue; splitting the kinds keeps each kernel's
// register footprint to that of one recursion.
template <int KIND>
__global__ __launch_bounds__(WG) void bt_item_kernel(KArgs A)
{
    __shared__ int s_item;
    __shared__ int s_flag;
    __shared__ int64_t s_scan[NWAVE];
    double *ws = A.ws + (int64_t)blockIdx.x * A.ws_doubles;
    int *wsi = A.wsi + (int64_t)blockIdx.x * A.wsi_ints;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.queue + KIND, 1);
        __syncthreads();
        const int q = s_item;
        __syncthreads();
        if (q >= A.n_items) break;
        const int opt = A.sched[q];
        const Model md = A.models[opt];
        if (!md.valid) continue;
        if (KIND == KIND_PRICE0) price0_item(A, md, opt, ws);
        else side_item<KIND>(A, md, opt, ws, wsi, s_scan, &s_flag);
        __syncthreads();
    }
}

// Initialises results (NaN prices, zero counts, status) and the queue.
__global__ void bt_reset_kernel(const Model *models, int n, bt_result *out, int *queue)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4) queue[i] = 0;
    if (i < n) {
        const double nan = __builtin_nan("");
        bt_result r;
        r.ask = nan; r.bid = nan; r.price0 = nan;
        r.bp_total_ask = 0; r.bp_total_bid = 0;
        r.bp_max_ask = 0; r.bp_max_bid = 0;
        r.status = models[i].valid ? BT_OK : BT_EINVAL;
        r.reserved = 0;
        out[i] = r;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
thread_local int g_last_hip = 0;

#define HIPCHK(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) {                        \
            g_last_hip = (int)e_;                      \
            return BT_EHIP;                            \
        }                                              \
    } while (0)

// Derives the tree constants of Section 4.1 for one option; false if the
// option is invalid (see bt_params in bt.h).
bool derive(const bt_params &p, Model &m)
{
    std::memset(&m, 0, sizeof(m));
    m.valid = 0;
    if (!(p.N >= 1 && p.N <= BT_MAX_N)) return false;
    if (!(std::isfinite(p.S0) && std::isfinite(p.K) && std::isfinite(p.R) && std::isfinite(p.sigma) &&
          std::isfinite(p.T) && std::isfinite(p.k)))
        return false;
    if (!(p.S0 > 0.0 && p.K > 0.0 && p.sigma > 0.0 && p.T > 0.0 && p.k >= 0.0 && p.k < 1.0)) return false;
    if (p.payoff < 0 || p.payoff > 2) return false;
    if (p.payoff == BT_BULL && !(std::isfinite(p.K2) && p.K2 > p.K)) return false;
    if (p.flags & ~(uint32_t)(BT_F_EUROPEAN | BT_F_COST_AT_T0)) return false;
    const double dt = p.T / (double)p.N;
    const double sq = std::sqrt(dt);
    const double u = std::exp(p.sigma * sq);
    const double r = std::exp(p.R * dt);
    const double d = 1.0 / u;
    const double rho = 1.0 / r;
    if (!(d < r && r < u)) return false;
    m.S0 = p.S0; m.u = u; m.d = d; m.r = r; m.rho = rho;
    m.p = (r - d) / (u - d);
    m.K = p.K; m.K2 = p.K2; m.k = p.k; m.sq = sq; m.dt = dt;
    m.N = p.N; m.payoff = p.payoff; m.flags = p.flags;
    m.valid = 1;
    return true;
}

}  // namespace

struct bt_book {
    int device = 0;
    int n = 0, n_max = 0, n_items = 0;
    int64_t nodes = 0;
    int grid = 0;
    int level_factor = 4;
    int64_t pool_doubles = 0;
    Model *d_models = nullptr;
    int *d_sched = nullptr;
    int *d_queue = nullptr;
    double *d_ws = nullptr;
    int *d_wsi = nullptr;
    KArgs args{};
    bool timing = false;
    std::vector<hipEvent_t> events;  // BT_NUM_KERNELS + 1 per timed call
    std::vector<bt_params> params;   // host copy, for re-pricing on overflow
    bt_tune tune{};
};

namespace {

void book_free(bt_book *b)
{
    if (!b) return;
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    b->events.clear();
    if (b->d_models) (void)hipFree(b->d_models);
    if (b->d_sched) (void)hipFree(b->d_sched);
    if (b->d_queue) (void)hipFree(b->d_queue);
    if (b->d_ws) (void)hipFree(b->d_ws);
    if (b->d_wsi) (void)hipFree(b->d_wsi);
    b->d_models = nullptr; b->d_sched = nullptr; b->d_queue = nullptr;
    b->d_ws = nullptr; b->d_wsi = nullptr;
}

int book_build(bt_book *b, const bt_params *h, int n, const bt_tune *tune)
{
    std::vector<Model> models(n);
    int n_max = 1;
    int64_t nodes = 0;
    for (int i = 0; i < n; i++) {
        if (derive(h[i], models[i])) {
            n_max = std::max(n_max, (int)h[i].N);
            nodes += (int64_t)(h[i].N + 1) * (h[i].N + 2) / 2;
        }
    }
    // options with valid parameters, longest tree first (one queue per kind)
    std::vector<int> sched;
    sched.reserve(n);
    for (int i = 0; i < n; i++)
        if (models[i].valid) sched.push_back(i);
    std::stable_sort(sched.begin(), sched.end(), [&](int x, int y) { return models[x].N > models[y].N; });

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    int wpc = (tune && tune->wgs_per_cu > 0) ? tune->wgs_per_cu : 2;
    int lf = (tune && tune->level_factor > 0) ? tune->level_factor : 8;
    int64_t pool = (tune && tune->pool_points > 0) ? (int64_t)tune->pool_points * 3 : (int64_t)1 << 20;
    int grid = std::max(1, std::min<int>((int)sched.size(), prop.multiProcessorCount * wpc));

    const int64_t nodes_cap = n_max + 2;
    const int64_t lcapd = (int64_t)lf * nodes_cap * 3 + nodes_cap;
    const Caps sc = small_caps();
    KArgs a{};
    a.oStab = 0;
    a.oL0 = ((2 * (int64_t)n_max + 3 + 31) / 32) * 32;
    a.oL1 = a.oL0 + ((lcapd + 31) / 32) * 32;
    a.oSmall = a.oL1 + ((lcapd + 31) / 32) * 32;
    a.oPool = a.oSmall + ((sc.total * WG + 31) / 32) * 32;
    a.ws_doubles = a.oPool + ((pool + 31) / 32) * 32;
    a.wsi_ints = ((4 * nodes_cap + 63) / 64) * 64;
    a.lcapd = lcapd;
    a.pool = pool;
    a.n_max = n_max;
    a.n_items = (int)sched.size();

    b->timing = tune && (tune->flags & BT_TUNE_TIMING);
    b->params.assign(h, h + n);
    if (tune) b->tune = *tune;
    b->device = dev;
    b->n = n; b->n_max = n_max; b->nodes = nodes; b->n_items = (int)sched.size();
    b->grid = grid; b->level_factor = lf; b->pool_doubles = pool;
    if (hipMalloc(&b->d_models, sizeof(Model) * n) != hipSuccess ||
        hipMalloc(&b->d_sched, sizeof(int) * std::max<size_t>(1, sched.size())) != hipSuccess ||
        hipMalloc(&b->d_queue, sizeof(int) * 64) != hipSuccess ||
        hipMalloc(&b->d_ws, sizeof(double) * a.ws_doubles * grid) != hipSuccess ||
        hipMalloc(&b->d_wsi, sizeof(int) * a.wsi_ints * grid) != hipSuccess) {
        (void)hipGetLastError();
        book_free(b);
        return BT_ENOMEM;
    }
    HIPCHK(hipMemcpy(b->d_models, models.data(), sizeof(Model) * n, hipMemcpyHostToDevice));
    if (!sched.empty()) HIPCHK(hipMemcpy(b->d_sched, sched.data(), sizeof(int) * sched.size(), hipMemcpyHostToDevice));
    a.models = b->d_models;
    a.sched = b->d_sched;
    a.queue = b->d_queue;
    a.ws = b->d_ws;
    a.wsi = b->d_wsi;
    b->args = a;
    return BT_OK;
}

}  // namespace

extern "C" {

int bt_book_create(const bt_params *h_params, int32_t n, const bt_tune *tune, bt_book **out)
{
    if (!out) return BT_EINVAL;
    *out = nullptr;
    if (!h_params || n < 1) return BT_EINVAL;
    bt_book *b = new (std::nothrow) bt_book();
    if (!b) return BT_ENOMEM;
    int rc = book_build(b, h_params, n, tune);
    if (rc != BT_OK) {
        book_free(b);
        delete b;
        return rc;
    }
    *out = b;
    return BT_OK;
}

int bt_book_info(const bt_book *book, int32_t *n, int32_t *n_max, int64_t *nodes)
{
    if (!book) return BT_EINVAL;
    if (n) *n = book->n;
    if (n_max) *n_max = book->n_max;
    if (nodes) *nodes = book->nodes;
    return BT_OK;
}

int bt_book_price(bt_book *book, bt_result *d_out, void *stream)
{
    if (!book || !d_out) return BT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    KArgs a = book->args;
    a.out = d_out;
    const int nb = (book->n + 255) / 256;
    hipEvent_t ev[BT_NUM_KERNELS + 1];
    if (book->timing) {
        for (int i = 0; i <= BT_NUM_KERNELS; i++) HIPCHK(hipEventCreate(&ev[i]));
        for (int i = 0; i <= BT_NUM_KERNELS; i++) book->events.push_back(ev[i]);
        HIPCHK(hipEventRecord(ev[0], s));
    }
    hipLaunchKernelGGL(bt_reset_kernel, dim3(nb), dim3(256), 0, s, book->d_models, book->n, d_out, book->d_queue);
    HIPCHK(hipGetLastError());
    if (book->timing) HIPCHK(hipEventRecord(ev[1], s));
    if (book->n_items > 0) {
        hipLaunchKernelGGL(bt_item_kernel<KIND_BID>, dim3(book->grid), dim3(WG), 0, s, a);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[2], s));
    if (book->n_items > 0) {
        hipLaunchKernelGGL(bt_item_kernel<KIND_ASK>, dim3(book->grid), dim3(WG), 0, s, a);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[3], s));
    if (book->n_items > 0) {
        hipLaunchKernelGGL(bt_item_kernel<KIND_PRICE0>, dim3(book->grid), dim3(WG), 0, s, a);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[4], s));
    return BT_OK;
}

int bt_book_price_grad(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream)
{
    (void)book; (void)d_out; (void)d_grad; (void)stream;
    return BT_ENOSUPP;
}

int bt_book_resolve_overflow(bt_book *book, bt_result *d_out, void *stream, int32_t *remaining)
{
    if (!book || !d_out) return BT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    std::vector<bt_result> res(book->n);
    HIPCHK(hipMemcpy(res.data(), d_out, sizeof(bt_result) * book->n, hipMemcpyDeviceToHost));
    std::vector<int> idx;
    for (int i = 0; i < book->n; i++)
        if (res[i].status == BT_EOVERFLOW) idx.push_back(i);
    int base_lf = book->tune.level_factor > 0 ? book->tune.level_factor : 8;
    int base_pool = book->tune.pool_points > 0 ? book->tune.pool_points : (1 << 20) / 3;
    for (int mult = 4; !idx.empty() && mult <= 1024; mult *= 4) {
        std::vector<bt_params> sub;
        for (int i : idx) sub.push_back(book->params[i]);
        bt_tune t = book->tune;
        t.flags = 0;
        t.level_factor = base_lf * mult;
        t.pool_points = (int32_t)std::min<int64_t>((int64_t)base_pool * mult, (int64_t)1 << 28);
        t.wgs_per_cu = 1;
        bt_book *sb = nullptr;
        int rc = bt_book_create(sub.data(), (int32_t)sub.size(), &t, &sb);
        if (rc != BT_OK) return rc;
        bt_result *d_sub = nullptr;
        if (hipMalloc(&d_sub, sizeof(bt_result) * sub.size()) != hipSuccess) {
            bt_book_destroy(sb);
            return BT_ENOMEM;
        }
        rc = bt_book_price(sb, d_sub, stream);
        std::vector<bt_result> sres(sub.size());
        if (rc == BT_OK) {
            hipError_t e = hipMemcpyAsync(sres.data(), d_sub, sizeof(bt_result) * sub.size(), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { g_last_hip = (int)e; rc = BT_EHIP; }
        }
        (void)hipFree(d_sub);
        bt_book_destroy(sb);
        if (rc != BT_OK) return rc;
        std::vector<int> still;
        for (size_t j = 0; j < idx.size(); j++) {
            res[idx[j]] = sres[j];
            if (sres[j].status == BT_EOVERFLOW) still.push_back(idx[j]);
        }
        idx.swap(still);
    }
    HIPCHK(hipMemcpyAsync(d_out, res.data(), sizeof(bt_result) * book->n, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (remaining) *remaining = (int32_t)idx.size();
    return BT_OK;
}

int bt_book_timings(bt_book *book, double *ms, int32_t *calls)
{
    if (!book || !ms) return BT_EINVAL;
    if (!book->timing) return BT_ENOSUPP;
    for (int i = 0; i < BT_NUM_KERNELS; i++) ms[i] = 0.0;
    const size_t per = BT_NUM_KERNELS + 1;
    const size_t nc = book->events.size() / per;
    int rc = BT_OK;
    for (size_t c = 0; c < nc; c++) {
        hipEvent_t *e = &book->events[c * per];
        if (hipEventSynchronize(e[BT_NUM_KERNELS]) != hipSuccess) rc = BT_EHIP;
        for (int i = 0; i < BT_NUM_KERNELS && rc == BT_OK; i++) {
            float t = 0.0f;
            hipError_t err = hipEventElapsedTime(&t, e[i], e[i + 1]);
            if (err != hipSuccess) { g_last_hip = (int)err; rc = BT_EHIP; }
            ms[i] += t;
        }
    }
    for (hipEvent_t e : book->events) (void)hipEventDestroy(e);
    book->events.clear();
    if (calls) *calls = (int32_t)nc;
    return rc;
}

void bt_book_destroy(bt_book *book)
{
    if (!book) return;
    (void)hipDeviceSynchronize();
    book_free(book);
    delete book;
}

int bt_price(const bt_params *p, bt_result *out)
{
    if (!p || !out) return BT_EINVAL;
    thread_local bt_book *cache = nullptr;
    thread_local int cache_nmax = 0;
    thread_local bt_result *d_res = nullptr;
    Model m;
    bool ok = derive(*p, m);
    int N = ok ? p->N : 1;
    if (!cache || N > cache_nmax || !ok) {
        if (cache) { bt_book_destroy(cache); cache = nullptr; }
        int rc = bt_book_create(p, 1, nullptr, &cache);
        if (rc != BT_OK) return rc;
        cache_nmax = cache->n_max;
        if (!d_res) HIPCHK(hipMalloc(&d_res, sizeof(bt_result)));
    } else {
        // reuse the cached buffers: new constants, same schedule shape
        HIPCHK(hipMemcpy(cache->d_models, &m, sizeof(Model), hipMemcpyHostToDevice));
    }
    int rc = bt_book_price(cache, d_res, nullptr);
    if (rc != BT_OK) return rc;
    HIPCHK(hipMemcpy(out, d_res, sizeof(bt_result), hipMemcpyDeviceToHost));
    return BT_OK;
}

int bt_model_constants(const bt_params *p, double *u, double *d, double *r, double *rho, double *pu)
{
    if (!p) return BT_EINVAL;
    Model m;
    if (!derive(*p, m)) return BT_EINVAL;
    if (u) *u = m.u;
    if (d) *d = m.d;
    if (r) *r = m.r;
    if (rho) *rho = m.rho;
    if (pu) *pu = m.p;
    return BT_OK;
}

const char *bt_strerror(int code)
{
    switch (code) {
    case BT_OK: return "success";
    case BT_EINVAL: return "invalid argument or option parameters";
    case BT_ENOMEM: return "out of memory";
    case BT_EHIP: return "HIP runtime error";
    case BT_EOVERFLOW: return "tree level exceeded the work buffers";
    case BT_ENOSUPP: return "not supported";
    default: return "unknown error";
    }
}

int bt_version(void) { return BT_VERSION; }

int bt_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
