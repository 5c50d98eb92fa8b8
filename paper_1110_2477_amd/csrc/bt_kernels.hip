// bt_kernels.hip -- gfx950 kernels of libbtprice and the C ABI around them.
//
// Seller (ask) and buyer (bid) recursions of Section 3 on the tree of
// Section 4.1.  Every tree side (option x party) is swept from level N+1 to
// the root in bands of `band` levels (a tuning field, at most BAND).  A band
// is cut into column blocks of WG - band output columns; the workgroup that
// owns a block also recomputes the halo of up to band-1 columns to its right
// that its trapezoid needs, so
// the blocks of a band are independent (the block/region partition of
// Section 4.2, with the region that would wait for a neighbour recomputed
// instead).  Consecutive bands are separated by kernel boundaries.  Band
// tasks of all tree sides of a book are handed to persistent workgroups from
// one counter per (launch, party).  The tree sides are aligned at the root:
// a tree side of nb bands runs its band r in launch r + nbands_max - nb, so
// every tree side ends in the last launch.  Nodes grow toward the root, so
// the expensive bands of trees of different N run side by side instead of
// one after another.
//
// Inside a block one lane owns one column; a level's records are packed
// variable-length PWL functions in per-workgroup buffers, the band's input
// and output levels live in per-tree-side buffers.  Node temporaries live in
// an interleaved per-lane area (coalesced across the wave); nodes with many
// breakpoints are collected per level and computed one per wavefront by the
// cooperative path of bt_wave.hpp.
//
// The zero-cost recursion runs in its own persistent kernel, one workgroup
// per option.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <functional>
#include <mutex>

#include "../../include/bt.h"
#include "bt_device.hpp"
#include "bt_wave.hpp"
#include "bt_adjoint.hpp"

using namespace bt;

namespace {

constexpr int BAND = 32;                   // default (and largest) levels per band
constexpr int MIN_BAND = 2;
constexpr int DEFAULT_LEVEL_FACTOR = 32;   // breakpoints per node the band buffers hold
constexpr int64_t DEFAULT_POOL_POINTS = (int64_t)1 << 18;   // per-workgroup pool, in breakpoints
constexpr int64_t MIN_PRIVATE_POINTS = (int64_t)1 << 16;    // floor of a private level, in breakpoints
constexpr int64_t DEFAULT_ARENA_DOUBLES = (int64_t)1 << 28;  // floor of one party's big-node arena
constexpr int64_t MAX_ARENA_DOUBLES = (int64_t)1 << 32;      // ceiling of the arena estimate (32 GiB)

// One tree side: option `opt`, party `side` (0 seller, 1 buyer); offsets of
// its two band-boundary level buffers (doubles) and index arrays (ints).
struct Item {
    int opt, side, N, nbands;
    int64_t lbuf, lcap;     // doubles: two buffers of lcap each at lbuf
    int64_t ibuf;           // ints: off[2][N+2], cnt[2][N+2]
    int64_t ctr;            // index of the first of nbands+1 fill counters
};

struct Task {
    int item, block;
};

struct KArgs {
    const Model *models;
    const Item *items;
    const Task *tasks;
    const int *task_lo;     // tasks of (launch L, side s): [task_lo, task_hi) at index 2L+s
    const int *task_hi;
    int *band_ctr;          // persistent-workgroup counters, [2 * nbands_max]
    unsigned long long *fill;   // band-buffer fill counters
    int *failed;            // per item
    int n_opts, n_items, nbands_max;
    int band;               // levels per band (a block has WG - band output columns)
    bt_result *out;
    double *lvl;            // tree-side band buffers
    int *lvli;
    double *ws;             // per workgroup: private levels, Stab, small area, pool
    int64_t ws_doubles;
    int *wsi;               // per workgroup: private level index arrays
    int64_t wsi_ints;
    int64_t ws_side, wsi_side;  // offset of the seller's (0) and buyer's (1) workspaces
    double *wsp;            // per workgroup of the zero-cost kernel: stock table, two levels
    int64_t p0_doubles, p0_stab;
    int64_t pcap;           // doubles per private level buffer
    int64_t pool;           // doubles in the pool
    int64_t oStab, oP0, oP1, oSmall, oPool;
    int *p0_queue;
    const int *p0_sched;
    const int *p0_count;    // number of options in p0_sched (device memory)
    bt_grad *grad;          // Greeks output (dual-number launches only)
    bt_hedge *hedge;        // holdings at t = 0 (or nullptr)
    unsigned char *exmap;   // exercise maps (or nullptr): option i's from exoff[i]
    const int64_t *exoff;   // n + 1 byte offsets
    double *arena;          // temporaries of big nodes that outgrow a wave's pool slice
    int64_t arena_cap[2];   // doubles of the seller's (0) and the buyer's (1) arena
    int64_t arena_base[2];  // their offsets in `arena` (the buyer's follows the seller's)
    unsigned long long *arena_ctr;  // bump counters, one per (band, party) launch
};

// Doubles of pool a wave needs for one cooperative node update whose
// children hold M points in all (high-water mark measured on the host at
// about 54 M for the buyer's update; the margin covers the rest).
__device__ __forceinline__ int64_t big_need(int M, int nt)
{
    return (((int64_t)64 * M + 4096) * nt + 31) & ~(int64_t)31;
}

// Takes n doubles of the arena for one wave (all lanes call; uniform
// result); nullptr when the arena is exhausted.
__device__ __forceinline__ double *arena_take(const KArgs &A, int ctr, int64_t n)
{
    unsigned long long pos = 0;
    if ((threadIdx.x & 63) == 0) pos = atomicAdd(A.arena_ctr + ctr, (unsigned long long)n);
    pos = __shfl(pos, 0, 64);
    if ((int64_t)pos + n > A.arena_cap[ctr & 1]) return nullptr;
    return A.arena + A.arena_base[ctr & 1] + pos;
}

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

template <typename T>
__device__ __forceinline__ View<T> record_view(const T *L, int64_t off, int m)
{
    return View<T>{L + off + 1, L + off + 2, L + off, m, 3};
}

template <typename T>
__device__ __forceinline__ void write_record(T *dst, const Arr<T> &z, int m)
{
    dst[0] = z.S(0);
    constexpr int B = pwl_group<T>();   // a group's loads before its stores
    for (int j0 = 0; j0 < m; j0 += B) {
        T x[B], v[B], sl[B];
#pragma unroll
        for (int u = 0; u < B; u++)
            if (j0 + u < m) { x[u] = z.X(j0 + u); v[u] = z.V(j0 + u); sl[u] = z.S(j0 + u + 1); }
#pragma unroll
        for (int u = 0; u < B; u++)
            if (j0 + u < m) { dst[1 + 3 * (j0 + u)] = x[u]; dst[2 + 3 * (j0 + u)] = v[u]; dst[3 + 3 * (j0 + u)] = sl[u]; }
    }
}

// Stock lattice S0 u^j for j = -(N+1)..N+1 (Section 4.1), by binary powering.
__device__ void stock_table(const Model &md, double *Stab)
{
    const int N = md.N;
    for (int idx = threadIdx.x; idx < 2 * N + 3; idx += WG) {
        int j = idx - (N + 1);
        double f = j >= 0 ? upow(md.u, j) : upow(md.d, -j);
        Stab[idx] = md.S0 * f;
    }
}

// Level N+1 of every tree side: the liquidation value y^- S^a - y^+ S^b
// (payoff (0, 0), Section 4.1), record [-(1+k) S, 0, 0, -(1-k) S], in band
// buffer 0.
template <typename T>
__global__ void bt_init_kernel(KArgs A)
{
  for (int it = blockIdx.y; it < A.n_items; it += gridDim.y) {
    const Item I = A.items[it];
    if (I.opt < 0) continue;   // unused slot of a batch planned on the device
    const Model md = A.models[I.opt];
    const Inputs<T> in = inputs_of(md, T{});
    const int N = I.N;
    T *L = (T *)(A.lvl + I.lbuf);
    int *off = A.lvli + I.ibuf, *cnt = off + 2 * (int64_t)(N + 2);
    const T one = mk<T>(1.0);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c <= N + 1; c += gridDim.x * blockDim.x) {
        const T S = stock_at(in, 2 * c - (N + 1));
        const T Sa = (one + in.k) * S, Sb = (one - in.k) * S;
        T *r = L + 4 * (int64_t)c;
        r[0] = -Sa; r[1] = mk<T>(0.0); r[2] = mk<T>(0.0); r[3] = -Sb;
        off[c] = 4 * c;
        cnt[c] = 1;
    }
  }
}

// One band task of launch `launch`: block `blk` of tree side `item`, whose
// band that launch runs.
// s_chunk / s_chunk_cap: each wave's arena chunk (kept for the whole launch
// and reused by the wave's later big nodes; grown when a node needs more).
template <int SIDE, typename T, bool EX = false>
__device__ __forceinline__ void band_task(const KArgs &A, int launch, int item, int blk, int64_t *sh, int *sflag,
                          double **s_chunk, int64_t *s_chunk_cap, T *s_win)
{
    constexpr int NT = sizeof(T) / sizeof(double);
    __shared__ int sbig[WG];
    __shared__ unsigned long long sloff;
    __shared__ unsigned long long sbase;
    const int tid = threadIdx.x;
    const Item I = A.items[item];
    const Model md = A.models[I.opt];
    const Inputs<T> in = inputs_of(md, T{});
    const int N = I.N;
    const int r = launch - (A.nbands_max - I.nbands);   // the tree side's band
    const int band = A.band, block_cols = WG - band;
    const int t_top = N - r * band;
    const int t_bot = t_top - band + 1 > 0 ? t_top - band + 1 : 0;
    const int c0 = blk * block_cols;
    const int c1 = min(c0 + block_cols, t_bot + 1);
    const bool last = c1 == t_bot + 1;

    // the two parties run concurrently, each on a workspace of its own
    double *ws = A.ws + SIDE * A.ws_side + (int64_t)blockIdx.x * A.ws_doubles;
    int *wsi = A.wsi + SIDE * A.wsi_side + (int64_t)blockIdx.x * A.wsi_ints;
    T *Stab = (T *)(ws + A.oStab);
    T *Pb[2] = {(T *)(ws + A.oP0), (T *)(ws + A.oP1)};
    const int64_t pcap = A.pcap / NT;        // numbers per private level
    int *poff[2] = {wsi, wsi + WG + 1};
    int *pcnt[2] = {wsi + 2 * (WG + 1), wsi + 3 * (WG + 1)};
    T *small = (T *)(ws + A.oSmall);
    double *pool = ws + A.oPool;
    // band-boundary buffers of this tree side
    const int64_t NN = N + 2;
    const int64_t lcap = I.lcap / NT;        // numbers per band buffer
    const T *Lin = (const T *)(A.lvl + I.lbuf + (int64_t)(r & 1) * I.lcap);
    T *Lout = (T *)(A.lvl + I.lbuf + (int64_t)((r + 1) & 1) * I.lcap);
    const int *offin = A.lvli + I.ibuf + (int64_t)(r & 1) * NN;
    const int *cntin = A.lvli + I.ibuf + 2 * NN + (int64_t)(r & 1) * NN;
    int *offout = A.lvli + I.ibuf + (int64_t)((r + 1) & 1) * NN;
    int *cntout = A.lvli + I.ibuf + 2 * NN + (int64_t)((r + 1) & 1) * NN;

    // stock prices of the lattice indices this block touches:
    // j = 2c - t for c in [c0, c0 + WG], t in [t_bot, t_top]
    const int jlo = 2 * c0 - t_top, jhi = 2 * (c0 + WG) - t_bot;
    for (int j = jlo + tid; j <= jhi; j += WG) Stab[j - jlo] = stock_at(in, j);
    if (tid == 0) *sflag = 0;
    __syncthreads();

    const Caps sc = small_caps();
    const bool euro = (md.flags & F_EUROPEAN) != 0;
    int64_t bp_sum = 0;
    int bp_max = 0;
    bool fatal = false;
    int cur = 0;
    for (int t = t_top; t >= t_bot && !fatal; t--) {
        const T kt = (t >= 1 || (md.flags & F_COST_AT_T0)) ? in.k : mk<T>(0.0);
        const bool exercise = !(euro && t < N);
        const int right = last ? t + 1 : min(c1 + (t - t_bot), t + 1);  // columns [c0, right)
        // children: the band's input level, or the previous private level
        const bool first = t == t_top;
        const T *Lc = first ? Lin : Pb[cur ^ 1];
        const int *offc = first ? offin + c0 : poff[cur ^ 1];
        const int *cntc = first ? cntin + c0 : pcnt[cur ^ 1];
        T *Ln = Pb[cur];
        int *offn = poff[cur], *cntn = pcnt[cur];
        const int i = tid;            // column c0 + i
        const int c = c0 + i;
        const bool act = c < right;
        View<T> Zu{}, Zd{};
        T S = mk<T>(0.0), xi = mk<T>(0.0), ze = mk<T>(0.0);
        int M = 0;
        if (act) {
            Zd = record_view(Lc, offc[i], cntc[i]);
            Zu = record_view(Lc, offc[i + 1], cntc[i + 1]);
            M = cntc[i] + cntc[i + 1];
            S = Stab[2 * c - t - jlo];
            payoff(md, in, S, xi, ze);
        }
        const bool owned = c < c1 || last;
        Arr<T> Z{};
        int mz = 0;
        bool big = act && M > SMALL_CAP;
        // exercise map (EX): node (t, c) of the party's plane
        int64_t exi = 0;
        if constexpr (EX) exi = A.exoff[I.opt] + (int64_t)SIDE * ((int64_t)(N + 1) * (N + 2) / 2) + (int64_t)t * (t + 1) / 2;
        if (act && !big) {
            int exf = 0;
            mz = node_update<SIDE, T>(Zu, Zd, S, kt, in.rho, xi, ze, exercise, small + tid, WG, sc, &Z,
                                      EX ? &exf : nullptr);
            big = mz < 0;
            if constexpr (EX) {
                if (!big && owned) A.exmap[exi + c] = (unsigned char)exf;
            }
        }
        // one scan for the record sizes (low 40 bits) and the big-node count
        const int64_t sz = (act && !big) ? 3 * (int64_t)mz + 1 : 0;
        const int64_t LOW = ((int64_t)1 << 40) - 1;
        int64_t tot;
        const int64_t ex = block_scan(sz + (big ? ((int64_t)1 << 40) : 0), &tot, sh);
        const int64_t nbig = tot >> 40, bix = ex >> 40, exs = ex & LOW;
        tot &= LOW;
        if (tot > pcap) {
            fatal = true;
        } else if (sz) {
            write_record(Ln + exs, Z, mz);
            offn[i] = (int)exs;
            cntn[i] = mz;
            if (owned) {
                const int bp = (mz == 1 && val(Z.S(0)) == val(Z.S(1))) ? 0 : mz;
                bp_sum += bp;
                bp_max = bp > bp_max ? bp : bp_max;
            }
        }
        int64_t loff = tot;
        if (nbig > 0 && !fatal) {
            if (big) sbig[bix] = i;
            if (tid == 0) sloff = (unsigned long long)loff;
            if (tid < NWAVE) bt_help[tid].state = 0;
            __syncthreads();
            const int w = tid >> 6, lane = tid & 63;
            // binary64 buyer: the waves with the two heaviest loads of big
            // nodes (children's points summed over the nodes each takes) get
            // the help of the two lightest -- a wave without a node at once,
            // one with nodes once they are done -- for parts of their
            // envelopes (bt_wave.hpp, SweepHelp; the mailbox is the helped
            // wave's): the load of rank r < NWAVE / 2 is helped by the one of
            // rank NWAVE - 1 - r
            int help = -1, helps = -1;
            if constexpr (SIDE == 1 && NT == 1) {
                static_assert(NWAVE == 4, "the pairing below is written for four waves");
                // loads of the four waves, one pass over the nodes (the lanes
                // take the nodes, a wave-wide sum per residue)
                int64_t ld[NWAVE] = {0, 0, 0, 0};
                for (int b0 = 0; b0 < (int)nbig; b0 += 64) {
                    const int b = b0 + lane;
                    const int64_t Mb = b < (int)nbig ? (int64_t)(cntc[sbig[b]] + cntc[sbig[b] + 1]) : 0;
#pragma unroll
                    for (int v = 0; v < NWAVE; v++) {
                        int64_t x = (b & 3) == v ? Mb : 0;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
                        ld[v] += x;
                    }
                }
                int rk[NWAVE];
#pragma unroll
                for (int v = 0; v < NWAVE; v++) {
                    int r = 0;
#pragma unroll
                    for (int o = 0; o < NWAVE; o++) r += (ld[o] > ld[v] || (ld[o] == ld[v] && o < v)) ? 1 : 0;
                    rk[v] = r;
                }
                const int rw = rk[w];
                if (rw < NWAVE / 2) {
                    help = w;
                } else {
#pragma unroll
                    for (int v = 0; v < NWAVE; v++)
                        if (rk[v] == NWAVE - 1 - rw) helps = v;
                }
            }
            const int64_t slice = A.pool / NWAVE;
            double *chunk = s_chunk[w];
            int64_t chunk_cap = s_chunk_cap[w];
            for (int bi = w; bi < (int)nbig; bi += NWAVE) {
                const int ii = sbig[bi];
                const int cc = c0 + ii;
                const View<T> Zd2 = record_view(Lc, offc[ii], cntc[ii]);
                const View<T> Zu2 = record_view(Lc, offc[ii + 1], cntc[ii + 1]);
                const T S2 = Stab[2 * cc - t - jlo];
                T xi2, ze2;
                payoff(md, in, S2, xi2, ze2);
                // the wave's pool slice when the node fits, else the arena;
                // a node that outgrows its slice is redone in the arena
                const int64_t need = big_need(Zu2.m + Zd2.m, NT);
                Arr<T> Zb;
                int mzb = -1, exf2 = 0;
#pragma unroll 1
                for (int attempt = need > slice ? 1 : 0; attempt < 2 && mzb < 0; attempt++) {
                    double *tb = pool + w * slice;
                    int64_t tcap = slice;
                    if (attempt == 1) {
                        if (chunk_cap < need) {
                            // a quarter of headroom for the slow growth of a
                            // tree side's nodes over the band; doubling when
                            // a later node outgrows the chunk
                            const int64_t grow = ((need + need / 4) + 31) & ~(int64_t)31;
                            const int64_t take = grow > 2 * chunk_cap ? grow : 2 * chunk_cap;
                            double *p = arena_take(A, 2 * launch + SIDE, take);
                            if (!p) break;
                            chunk = p;
                            chunk_cap = take;
                        }
                        tb = chunk;
                        tcap = chunk_cap;
                    }
                    WaveTmp WT{tb, tcap, 0};
                    mzb = wave_node_update<SIDE, T>(Zu2, Zd2, S2, kt, in.rho, xi2, ze2, exercise, WT,
                                                    s_win + w * WaveLds<T>::NUMS, &Zb, EX ? &exf2 : nullptr, help);
                }
                if (mzb < 0) {
                    if (lane == 0) *sflag = 1;
                    continue;
                }
                const int64_t rec = 3 * (int64_t)mzb + 1;
                unsigned long long pos = 0;
                if (lane == 0) pos = atomicAdd(&sloff, (unsigned long long)rec);
                pos = __shfl(pos, 0, 64);
                if ((int64_t)pos + rec > pcap) {
                    if (lane == 0) *sflag = 1;
                    continue;
                }
                T *dst = Ln + pos;
                {
                    // several points per lane in flight: the loads of a
                    // group issue before its stores
                    constexpr int U = NT == 1 ? 4 : 1;
                    for (int j0 = 0; j0 < mzb; j0 += 64 * U) {
                        T x[U], v[U], sl[U];
#pragma unroll
                        for (int u = 0; u < U; u++) {
                            const int j = j0 + 64 * u + lane;
                            if (j < mzb) { x[u] = Zb.X(j); v[u] = Zb.V(j); sl[u] = Zb.S(j + 1); }
                        }
#pragma unroll
                        for (int u = 0; u < U; u++) {
                            const int j = j0 + 64 * u + lane;
                            if (j < mzb) { dst[1 + 3 * j] = x[u]; dst[2 + 3 * j] = v[u]; dst[3 + 3 * j] = sl[u]; }
                        }
                    }
                }
                if (lane == 0) {
                    dst[0] = Zb.S(0);
                    offn[ii] = (int)pos;
                    cntn[ii] = mzb;
                    if constexpr (EX) {
                        if (cc < c1 || last) A.exmap[exi + cc] = (unsigned char)exf2;
                    }
                    if (cc < c1 || last) {
                        const int bp = (mzb == 1 && val(Zb.S(0)) == val(Zb.S(1))) ? 0 : mzb;
                        bp_sum += bp;
                        bp_max = bp > bp_max ? bp : bp_max;
                    }
                }
            }
            if constexpr (SIDE == 1 && NT == 1) {
                if (help >= 0) help_post(help, 3);
                if (helps >= 0) sweep_helper(helps, (double *)(s_win + w * WaveLds<T>::NUMS));
            }
            if (lane == 0) {
                s_chunk[w] = chunk;
                s_chunk_cap[w] = chunk_cap;
            }
            __syncthreads();
            loff = (int64_t)sloff;
            if (*sflag) fatal = true;
        }
        __syncthreads();
        if (t == t_bot && !fatal) {
            // the band's output level (columns [c0, c1)) goes to the tree
            // side's band buffer; level 0 gives the price
            if (tid == 0) {
                sbase = atomicAdd(A.fill + I.ctr + r + 1, (unsigned long long)loff);
                if ((int64_t)sbase + loff > lcap) *sflag = 1;
            }
            __syncthreads();
            if (*sflag) {
                fatal = true;
            } else {
                const int64_t base = (int64_t)sbase;
                {
                    constexpr int U = NT == 1 ? 4 : 1;
                    for (int64_t q0 = 0; q0 < loff; q0 += (int64_t)WG * U) {
                        T r[U];
#pragma unroll
                        for (int u = 0; u < U; u++) {
                            const int64_t q = q0 + (int64_t)u * WG + tid;
                            if (q < loff) r[u] = Ln[q];
                        }
#pragma unroll
                        for (int u = 0; u < U; u++) {
                            const int64_t q = q0 + (int64_t)u * WG + tid;
                            if (q < loff) Lout[base + q] = r[u];
                        }
                    }
                }
                if (tid < c1 - c0) {
                    offout[c0 + tid] = (int)(base + offn[tid]);
                    cntout[c0 + tid] = cntn[tid];
                }
                if (t == 0 && tid == 0 && A.hedge) {
                    // the hedge from the root's children, in the (now idle)
                    // pool of this workgroup
                    const View<T> Zd0 = record_view(Lc, offc[0], cntc[0]);
                    const View<T> Zu0 = record_view(Lc, offc[1], cntc[1]);
                    const T S0 = Stab[-jlo];   // column 0 at t = 0
                    const T one = mk<T>(1.0);
                    const int hcap = (int)std::min<int64_t>((A.pool / NT - 1) / 3, INT32_MAX);
                    double lo = __builtin_nan(""), hi = __builtin_nan("");
                    if (!root_hedge<T>(Zu0, Zd0, in.rho, val((one + kt) * S0), val((one - kt) * S0), (T *)pool,
                                       hcap, &lo, &hi))
                        lo = hi = __builtin_nan("");
                    if (SIDE == 0) { A.hedge[I.opt].ask_lo = lo; A.hedge[I.opt].ask_hi = hi; }
                    else { A.hedge[I.opt].bid_lo = lo; A.hedge[I.opt].bid_hi = hi; }
                }
                if (t == 0 && tid == 0) {
                    const T root = eval(record_view(Ln, offn[0], cntn[0]), mk<T>(0.0));
                    const T price = SIDE == 0 ? root : -root;
                    if (SIDE == 0) A.out[I.opt].ask = val(price);
                    else A.out[I.opt].bid = val(price);
                    if constexpr (NT == 5) {
                        bt_grad4 &g = SIDE == 0 ? A.grad[I.opt].ask : A.grad[I.opt].bid;
                        g.dS0 = price.d[0]; g.dsigma = price.d[1]; g.dR = price.d[2]; g.dk = price.d[3];
                    }
                }
            }
        }
        cur ^= 1;
    }

    // breakpoint statistics of the owned columns
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
        bt_result &o = A.out[I.opt];
        if (fatal) {
            atomicMin(&o.status, BT_EOVERFLOW);
            atomicExch(A.failed + item, 1);
        } else {
            atomicAdd((unsigned long long *)(SIDE == 0 ? &o.bp_total_ask : &o.bp_total_bid),
                      (unsigned long long)ts);
            atomicMax(SIDE == 0 ? &o.bp_max_ask : &o.bp_max_bid, tm);
        }
    }
    __syncthreads();
}

// Launch r of one party: the bands of its tree sides that this launch runs
// (see the file header), on persistent workgroups.
template <int SIDE, typename T, bool EX = false>
__global__ __launch_bounds__(WG) void bt_band_kernel(KArgs A, int r)
{
    __shared__ int s_task, s_skip;
    __shared__ int s_flag;
    __shared__ int64_t s_scan[NWAVE];
    __shared__ double *s_chunk[NWAVE];
    __shared__ int64_t s_chunk_cap[NWAVE];
    __shared__ T s_win[NWAVE * WaveLds<T>::NUMS];   // MERGE windows of the cooperative path
    const int lo = A.task_lo[2 * r + SIDE], hi = A.task_hi[2 * r + SIDE];
    if (threadIdx.x < NWAVE) {
        s_chunk[threadIdx.x] = nullptr;
        s_chunk_cap[threadIdx.x] = 0;
    }
    for (;;) {
        if (threadIdx.x == 0) {
            const int q0 = lo + atomicAdd(A.band_ctr + 2 * r + SIDE, 1);
            s_task = q0;
            // a tree side whose earlier work overflowed is skipped (one read,
            // shared by the whole workgroup)
            s_skip = q0 < hi ? __hip_atomic_load(A.failed + A.tasks[q0].item, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : 0;
        }
        __syncthreads();
        const int q = s_task, skip = s_skip;
        __syncthreads();
        if (q >= hi) break;
        if (skip) continue;
        const Task tk = A.tasks[q];
        band_task<SIDE, T, EX>(A, r, tk.item, tk.block, s_scan, &s_flag, s_chunk, s_chunk_cap, s_win);
    }
}

// Zero-cost recursion (Section 3, Appendix): no extra level;
// V_N = max(xi + zeta S, 0), V_t = max(xi + zeta S, rho (p V_up + (1-p) V_dn))
// (European variant: V_t = continuation value).  One workgroup per option.
__device__ __forceinline__ void price0_item(const KArgs &A, const Model &md, int opt, double *ws)
{
    const int N = md.N;
    double *Stab = ws;
    double *V0 = ws + A.p0_stab, *V1 = ws + A.p0_stab + (N + 1);
    const Inputs<double> in = inputs_of(md, 0.0);
    stock_table(md, Stab);
    __syncthreads();
    const bool euro = (md.flags & F_EUROPEAN) != 0;
    for (int c = threadIdx.x; c <= N; c += WG) {
        double S = Stab[2 * c + 1], xi, ze;
        payoff(md, in, S, xi, ze);
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
            payoff(md, in, S, xi, ze);
            double P = xi + ze * S;
            if (P < 0.0) P = 0.0;
            nxt[c] = P > cont ? P : cont;
        }
        __syncthreads();
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (threadIdx.x == 0) A.out[opt].price0 = cur[0];
}

// The same recursion with the level in registers: lane l holds columns
// l + 256 m, m < J.  A node's upper child is the next lane's value (a DPP
// wave shift) or, for a wave's last lane, the first lane's value of the next
// wave (or of wave 0 at m + 1), which each wave's first lane leaves in LDS;
// two LDS buffers alternate by level, so one barrier per level suffices.
// Every node takes price0_item's operations in its order (the clamp of the
// exercise value at 0 is taken once per lattice index), so the bits agree.
constexpr int P0_JMAX = 80;   // levels of up to 256 * 80 nodes stay in registers

template <int J>
__device__ __forceinline__ void price0_regs(const KArgs &A, const Model &md, int opt, double *Ptab,
                                            double (*edge)[NWAVE][P0_JMAX])
{
    constexpr int CH = J < 8 ? J : 8;
    static_assert(J % CH == 0, "columns per lane in whole groups");
    const int N = md.N;
    const int l = threadIdx.x, w = l >> 6, ll = l & 63;
    const Inputs<double> in = inputs_of(md, 0.0);
    // the exercise value max(xi + zeta S, 0) depends on the lattice index
    // j = 2c - t alone: one table entry per j, computed as price0_item does
    for (int idx = l; idx < 2 * N + 3; idx += WG) {
        const int j = idx - (N + 1);
        double S = md.S0 * (j >= 0 ? upow(md.u, j) : upow(md.d, -j)), xi, ze;
        payoff(md, in, S, xi, ze);
        const double P = xi + ze * S;
        Ptab[idx] = P > 0.0 ? P : 0.0;
    }
    __syncthreads();
    const bool euro = (md.flags & F_EUROPEAN) != 0;
    double v[J];
#pragma unroll
    for (int m = 0; m < J; m++) {
        const int c = l + WG * m;
        v[m] = c <= N ? Ptab[2 * c + 1] : 0.0;
    }
    const double p = md.p, q = 1.0 - md.p, rho = md.rho;
    for (int t = N - 1; t >= 0; t--) {
        double(*eb)[P0_JMAX] = edge[t & 1];
        // columns in groups of CH; the next group's exercise values load
        // while the current group computes (the first group's before the
        // barrier)
        double Pn[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const int idx = 2 * (l + WG * k) - t + N + 1;
            Pn[k] = euro ? 0.0 : Ptab[idx < 2 * N + 2 ? idx : 2 * N + 2];
        }
        if (ll == 0) {
#pragma unroll
            for (int m = 0; m < J; m++)
                if (WG * m <= t + 1) eb[w][m] = v[m];
        }
        __syncthreads();
#pragma unroll
        for (int m0 = 0; m0 < J; m0 += CH) {
            double Pg[CH];
#pragma unroll
            for (int k = 0; k < CH; k++) Pg[k] = Pn[k];
            if (m0 + CH < J && WG * (m0 + CH) <= t && !euro) {
#pragma unroll
                for (int k = 0; k < CH; k++) {
                    const int idx = 2 * (l + WG * (m0 + CH + k)) - t + N + 1;
                    Pn[k] = Ptab[idx < 2 * N + 2 ? idx : 2 * N + 2];
                }
            }
            if (WG * m0 > t) continue;
            // the values past each wave's last lane, read together (every
            // lane of a wave reads the same word)
            double Eg[CH];
#pragma unroll
            for (int k = 0; k < CH; k++) {
                const int m = m0 + k;
                Eg[k] = w < NWAVE - 1 ? eb[w + 1][m] : (m + 1 < J ? eb[0][m + 1] : 0.0);
            }
#pragma unroll
            for (int k = 0; k < CH; k++) {
                const int m = m0 + k;
                double up = dpp_d<0x130>(0.0, v[m]);
                if (ll == 63) up = Eg[k];
                if (l + WG * m <= t) {
                    const double cont = rho * (p * up + q * v[m]);
                    v[m] = euro ? cont : (Pg[k] > cont ? Pg[k] : cont);
                }
            }
        }
    }
    if (l == 0) A.out[opt].price0 = v[0];
}

__global__ __launch_bounds__(WG) void bt_price0_kernel(KArgs A)
{
    __shared__ int s_item;
    __shared__ double s_edge[2][NWAVE][P0_JMAX];
    double *ws = A.wsp + (int64_t)blockIdx.x * A.p0_doubles;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.p0_queue, 1);
        __syncthreads();
        const int q = s_item;
        __syncthreads();
        if (q >= *A.p0_count) break;
        const int opt = A.p0_sched[q];
        const Model md = A.models[opt];
        const int n1 = md.N + 1;
        if (n1 <= WG * 4) price0_regs<4>(A, md, opt, ws, s_edge);
        else if (n1 <= WG * 16) price0_regs<16>(A, md, opt, ws, s_edge);
        else if (n1 <= WG * 40) price0_regs<40>(A, md, opt, ws, s_edge);
        else if (n1 <= WG * P0_JMAX) price0_regs<P0_JMAX>(A, md, opt, ws, s_edge);
        else price0_item(A, md, opt, ws);
        __syncthreads();
    }
}

// Initialises results (NaN prices, zero counts, status), queues, fill
// counters and failure flags.
__global__ void bt_reset_kernel(KArgs A, int64_t n_fill)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < A.n_opts; k += stride) {
        const double nan = __builtin_nan("");
        bt_result r;
        r.ask = nan; r.bid = nan; r.price0 = nan;
        r.bp_total_ask = 0; r.bp_total_bid = 0;
        r.bp_max_ask = 0; r.bp_max_bid = 0;
        r.status = A.models[k].valid ? BT_OK : BT_EINVAL;
        r.reserved = 0;
        A.out[k] = r;
        if (A.grad) {
            bt_grad g;
            g.ask.dS0 = g.ask.dsigma = g.ask.dR = g.ask.dk = nan;
            g.bid = g.ask;
            A.grad[k] = g;
        }
        if (A.hedge) {
            bt_hedge h;
            h.ask_lo = h.ask_hi = h.bid_lo = h.bid_hi = nan;
            A.hedge[k] = h;
        }
    }
    for (int64_t k = i; k < 2 * (int64_t)A.nbands_max; k += stride) {
        A.band_ctr[k] = 0;
        A.arena_ctr[k] = 0;
    }
    for (int64_t k = i; k < n_fill; k += stride) A.fill[k] = 0;
    for (int64_t k = i; k < A.n_items; k += stride) A.failed[k] = 0;
    if (i == 0) *A.p0_queue = 0;
}

// ---------------------------------------------------------------------------
// Reverse-mode Greeks (bt_price_adjoint_batch).  One workgroup sweeps one
// tree side at a time:
//   forward   levels N+1 .. 1 from the leaves, keeping the levels
//             t = N+1, N+1-s, N+1-2s, ... (s = ceil(sqrt(N+2))) as
//             checkpoints;
//   reverse   segment by segment from the root: the levels between a
//             checkpoint and the next lower one are recomputed from the
//             checkpoint, then the reverse steps t = lo .. hi-1 carry the
//             adjoint from level t to level t+1 (bt_adjoint.hpp); finally the
//             leaves' adjoint gives their stock prices' and the cost rate's
//             contributions.
// Nodes whose children hold at most ADJ_LANE_PTS points are stepped by one lane
// each; larger ones are queued and stepped by the first lane of a wave with
// that wave's large-node slot.  The adjoint of a child is the sum of what its
// two parents give it; parents of even and of odd columns run in two passes,
// so no two lanes add to one child at once and the sums have a fixed order.
// ---------------------------------------------------------------------------
// a lane steps nodes whose children hold up to ADJ_LANE_PTS points (stages
// of 2 ADJ_LANE_PTS + 16, tape of ADJ_LANE_TAPE entries)
constexpr int ADJ_LANE_PTS = 32;
constexpr int ADJ_LANE_TAPE = 2048;

struct AdjArgs {
    const Model *models;
    const int *order;       // options, longest tree first
    const int *count;       // number of options in `order`
    int *queue;             // [2]: next position per party
    bt_result *out;
    bt_grad *grad;
    double *ws;             // per workgroup, ws_doubles each
    int64_t ws_doubles;
    int *wsi;               // per workgroup, wsi_ints each
    int64_t wsi_ints;
    int Ncap, big_pts;      // largest N; largest child points of a queued node
    int64_t lwn;            // numbers per level slot (W0, W1, A0, A1)
    int64_t cp_nums, sg_nums;   // numbers of the checkpoint and segment regions
    int cp_max, sg_max;     // levels they index
    // offsets in a workgroup's doubles
    int64_t oStab, oSfac, oW0, oW1, oA0, oA1, oCP, oSG, oLane, oBig;
    int64_t lane_doubles, big_doubles;
    // offsets in a workgroup's ints: off/cnt of W0, W1, the checkpoints and
    // the segment levels ((N+2) each), then the checkpoint table
    int64_t iW0, iW1, iCP, iSG, iTab;
};

struct LevelRef {
    double *rec;
    int *off, *cnt;
};

// Scratch of one stepper (a lane's, or a wave's large-node slot).
struct Stepper {
    double *fwd;            // forward stages (doubles)
    Caps fcp;
    TN *tn;
    RevCaps rc;
    TapeEnt *ent;
    double *adj, *gd, *gu;
};

BTHD int64_t stepper_doubles(int stage_cap, int child_cap, int tape)
{
    const Caps f = make_caps(stage_cap, stage_cap, stage_cap, stage_cap, stage_cap);
    const RevCaps r = rev_caps(stage_cap, child_cap, tape);
    int64_t d = (f.total + 1) & ~(int64_t)1;
    d += 2 * r.tn;                                  // TN: 16 bytes each
    d += 3 * (int64_t)tape;                         // tape entries: 24 bytes each
    d += 3 * 2 * (int64_t)child_cap + 5 + tape;     // adj
    d += 2 * (3 * (int64_t)child_cap + 1);          // gd, gu
    return (d + 31) & ~(int64_t)31;
}

__device__ Stepper make_stepper(double *p, int stage_cap, int child_cap, int tape)
{
    Stepper S;
    S.fcp = make_caps(stage_cap, stage_cap, stage_cap, stage_cap, stage_cap);
    S.rc = rev_caps(stage_cap, child_cap, tape);
    S.fwd = p;
    p += (S.fcp.total + 1) & ~(int64_t)1;
    S.tn = (TN *)p;
    p += 2 * S.rc.tn;
    S.ent = (TapeEnt *)p;
    p += 3 * (int64_t)tape;
    S.adj = p;
    p += 3 * 2 * (int64_t)child_cap + 5 + tape;
    S.gd = p;
    p += 3 * (int64_t)child_cap + 1;
    S.gu = p;
    return S;
}

__device__ __forceinline__ View<double> level_view(const LevelRef &L, int c)
{
    const double *r = L.rec + L.off[c];
    return View<double>{r + 1, r + 2, r, L.cnt[c], 3};
}

// Level t (t+1 columns) from level `up` into `dst` (records from offset 0,
// at most cap numbers).  Returns the numbers written, or -1 on overflow
// (uniform over the workgroup).
template <int SIDE>
__device__ int64_t adj_fwd_level(const AdjArgs &A, const Model &md, int t, const double *Stab, const LevelRef &up,
                                 const LevelRef &dst, int64_t cap, const Stepper &lane, const Stepper &big,
                                 int64_t *bp_sum, int *bp_max, int64_t *sh, int *sbig, int64_t *srun, int *sflag)
{
    const int tid = threadIdx.x, w = tid >> 6, ln = tid & 63;
    const int N = md.N;
    const Inputs<double> in = inputs_of(md, 0.0);
    const double kt = (t >= 1 || (md.flags & F_COST_AT_T0)) ? md.k : 0.0;
    const bool ex = !((md.flags & F_EUROPEAN) && t < N);
    int64_t run = 0;
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int c0 = 0; c0 <= t; c0 += WG) {
        const int c = c0 + tid;
        const bool act = c <= t;
        int mz = 0;
        bool bigq = false;
        Arr<double> Z{};
        if (act) {
            const View<double> Zd = level_view(up, c), Zu = level_view(up, c + 1);
            if (Zd.m + Zu.m > ADJ_LANE_PTS) {
                bigq = true;
            } else {
                const double S = Stab[2 * c - t + N + 1];
                double xi, ze;
                payoff(md, in, S, xi, ze);
                mz = node_update<SIDE, double>(Zu, Zd, S, kt, md.rho, xi, ze, ex, lane.fwd, 1, lane.fcp, &Z);
                bigq = mz < 0;
            }
        }
        const int64_t sz = (act && !bigq) ? 3 * (int64_t)mz + 1 : 0;
        const int64_t LOW = ((int64_t)1 << 40) - 1;
        int64_t tot;
        const int64_t exs = block_scan(sz + (bigq ? ((int64_t)1 << 40) : 0), &tot, sh);
        const int nbig = (int)(tot >> 40), bix = (int)(exs >> 40);
        tot &= LOW;
        const int64_t pos = run + (exs & LOW);
        if (run + tot > cap) {
            if (tid == 0) *sflag = 1;
        } else if (sz) {
            double *d = dst.rec + pos;
            d[0] = Z.S(0);
            for (int j = 0; j < mz; j++) {
                d[1 + 3 * j] = Z.X(j);
                d[2 + 3 * j] = Z.V(j);
                d[3 + 3 * j] = Z.S(j + 1);
            }
            dst.off[c] = (int)pos;
            dst.cnt[c] = mz;
            const int bp = (mz == 1 && Z.S(0) == Z.S(1)) ? 0 : mz;
            *bp_sum += bp;
            *bp_max = bp > *bp_max ? bp : *bp_max;
        }
        if (bigq) sbig[bix] = c;
        if (tid == 0) *srun = run + tot;
        __syncthreads();
        if (*sflag) return -1;
        for (int bi = w; bi < nbig; bi += NWAVE) {
            if (ln != 0) continue;
            const int cc = sbig[bi];
            const View<double> Zd = level_view(up, cc), Zu = level_view(up, cc + 1);
            const double S = Stab[2 * cc - t + N + 1];
            double xi, ze;
            payoff(md, in, S, xi, ze);
            Arr<double> Zb;
            const int mb = (Zd.m + Zu.m <= A.big_pts)
                               ? node_update<SIDE, double>(Zu, Zd, S, kt, md.rho, xi, ze, ex, big.fwd, 1, big.fcp, &Zb)
                               : -1;
            if (mb < 0) { *sflag = 1; continue; }
            const int64_t rec = 3 * (int64_t)mb + 1;
            const int64_t p = (int64_t)atomicAdd((unsigned long long *)srun, (unsigned long long)rec);
            if (p + rec > cap) { *sflag = 1; continue; }
            double *d = dst.rec + p;
            d[0] = Zb.S(0);
            for (int j = 0; j < mb; j++) {
                d[1 + 3 * j] = Zb.X(j);
                d[2 + 3 * j] = Zb.V(j);
                d[3 + 3 * j] = Zb.S(j + 1);
            }
            dst.off[cc] = (int)p;
            dst.cnt[cc] = mb;
            const int bp = (mb == 1 && Zb.S(0) == Zb.S(1)) ? 0 : mb;
            *bp_sum += bp;
            *bp_max = bp > *bp_max ? bp : *bp_max;
        }
        __syncthreads();
        run = *srun;
        if (*sflag) return -1;
        __syncthreads();
    }
    return run;
}

// Greeks accumulators of one lane.
struct GAcc {
    double S0, sig, R, k;
};

// One reverse step of node (t, c): adds its children's adjoints into Anxt
// and its parameters' into g.  false when a capacity was too small.
template <int SIDE>
__device__ bool adj_node(const AdjArgs &A, const Model &md, int t, int c, const double *Stab, const double *Sfac,
                         const LevelRef &Lt, const LevelRef &Lc, const double *Acur, double *Anxt, const Stepper &st,
                         GAcc &g, double *price)
{
    const int N = md.N;
    const bool t0cost = (md.flags & F_COST_AT_T0) != 0;
    const double kt = (t >= 1 || t0cost) ? md.k : 0.0;
    const bool ex = !((md.flags & F_EUROPEAN) && t < N);
    const View<double> Zd = level_view(Lc, c), Zu = level_view(Lc, c + 1);
    const double S = Stab[2 * c - t + N + 1];
    const double *zbar = t >= 1 ? Acur + Lt.off[c] : nullptr;
    const int mz = t >= 1 ? Lt.cnt[c] : 0;
    double gp[3];
    if (node_reverse<SIDE>(md, Zd, Zu, S, kt, md.rho, ex, zbar, mz, st.rc, st.tn, threadIdx.x, st.ent, st.adj, st.gd,
                           st.gu, gp, price))
        return false;
    double *ad = Anxt + Lc.off[c], *au = Anxt + Lc.off[c + 1];
    for (int q = 0; q < 3 * Zd.m + 1; q++) ad[q] += st.gd[q];
    for (int q = 0; q < 3 * Zu.m + 1; q++) au[q] += st.gu[q];
    const int j = 2 * c - t;
    g.S0 += gp[0] * Sfac[j + N + 1];
    g.sig += gp[0] * (S * (double)j * md.sq);
    g.R += gp[2] * (-md.dt * md.rho);
    if (t >= 1 || t0cost) g.k += gp[1];
    return true;
}

// Reverse step of level t: Acur (adjoint of level t, layout Lt; unused at
// t = 0) to Anxt (adjoint of level t+1, layout Lc, `nn` numbers).  false
// when a node did not fit (uniform over the workgroup).
template <int SIDE>
__device__ bool adj_rev_level(const AdjArgs &A, const Model &md, int t, const double *Stab, const double *Sfac,
                              const LevelRef &Lt, const LevelRef &Lc, int64_t nn, const double *Acur, double *Anxt,
                              const Stepper &lane, const Stepper &big, GAcc &g, double *price, int64_t *sh, int *sbig,
                              int *sflag)
{
    const int tid = threadIdx.x, w = tid >> 6, ln = tid & 63;
    for (int64_t q = tid; q < nn; q += WG) Anxt[q] = 0.0;
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int par = 0; par < 2; par++) {
        for (int c0 = par; c0 <= t; c0 += 2 * WG) {
            const int c = c0 + 2 * tid;
            bool bigq = false;
            if (c <= t) {
                const int M = Lc.cnt[c] + Lc.cnt[c + 1];
                bigq = M > ADJ_LANE_PTS || !adj_node<SIDE>(A, md, t, c, Stab, Sfac, Lt, Lc, Acur, Anxt, lane, g, price);
            }
            int64_t tot;
            const int64_t bix = block_scan(bigq ? 1 : 0, &tot, sh);
            if (bigq) sbig[bix] = c;
            __syncthreads();
            for (int bi = w; bi < (int)tot; bi += NWAVE) {
                if (ln != 0) continue;
                const int cc = sbig[bi];
                const bool ok = Lc.cnt[cc] + Lc.cnt[cc + 1] <= A.big_pts &&
                                adj_node<SIDE>(A, md, t, cc, Stab, Sfac, Lt, Lc, Acur, Anxt, big, g, price);
                if (!ok) *sflag = 1;
            }
            __syncthreads();
            if (*sflag) return false;
        }
    }
    return true;
}

// Integer ceil(sqrt(x)) for x >= 1.
BTHD int isqrt_ceil(int x)
{
    int s = 1;
    while ((int64_t)s * s < x) s++;
    return s;
}

// Copies a level (records, offsets, counts of `ncol` columns, `nn` numbers)
// to dst.
__device__ void copy_level(const LevelRef &src, const LevelRef &dst, int ncol, int64_t nn)
{
    constexpr int U = 4;   // loads of a group issue before its stores
    for (int64_t q0 = 0; q0 < nn; q0 += (int64_t)WG * U) {
        double r[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t q = q0 + (int64_t)u * WG + threadIdx.x;
            if (q < nn) r[u] = src.rec[q];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t q = q0 + (int64_t)u * WG + threadIdx.x;
            if (q < nn) dst.rec[q] = r[u];
        }
    }
    for (int c = threadIdx.x; c < ncol; c += WG) {
        dst.off[c] = src.off[c];
        dst.cnt[c] = src.cnt[c];
    }
    __syncthreads();
}

template <int SIDE>
__device__ void adjoint_tree(const AdjArgs &A, int opt, int64_t *sh, int *sbig, int64_t *srun, int *sflag)
{
    const int tid = threadIdx.x, w = tid >> 6;
    const Model md = A.models[opt];
    const int N = md.N;
    double *ws = A.ws + (int64_t)blockIdx.x * A.ws_doubles;
    int *wsi = A.wsi + (int64_t)blockIdx.x * A.wsi_ints;
    double *Stab = ws + A.oStab, *Sfac = ws + A.oSfac;
    const Inputs<double> in = inputs_of(md, 0.0);
    for (int idx = tid; idx < 2 * N + 3; idx += WG) {
        const int j = idx - (N + 1);
        Sfac[idx] = j >= 0 ? upow(md.u, j) : upow(md.d, -j);
        Stab[idx] = stock_at(in, j);
    }
    __syncthreads();
    const int64_t NN = N + 2;
    LevelRef W[2] = {{ws + A.oW0, wsi + A.iW0, wsi + A.iW0 + NN}, {ws + A.oW1, wsi + A.iW1, wsi + A.iW1 + NN}};
    double *Abuf[2] = {ws + A.oA0, ws + A.oA1};
    // checkpoint table: per checkpoint, its record offset in the region;
    // then per segment level, its record offset
    int64_t *cp_base = (int64_t *)(wsi + A.iTab);
    int64_t *sg_base = cp_base + A.cp_max + 1;
    const Stepper lane = make_stepper(ws + A.oLane + (int64_t)tid * A.lane_doubles, 2 * ADJ_LANE_PTS + 16, ADJ_LANE_PTS,
                                      ADJ_LANE_TAPE);
    const Stepper big = make_stepper(ws + A.oBig + (int64_t)w * A.big_doubles, 2 * A.big_pts + 16, A.big_pts,
                                     40 * A.big_pts + 4096);
    const int s = isqrt_ceil(N + 2);
    const int ncp = N / s + 1;   // checkpoints t = N+1 - j s >= 1, j = 0 .. ncp-1
    const auto cp_level = [&](int j) {
        return LevelRef{ws + A.oCP + cp_base[j], wsi + A.iCP + 2 * NN * j, wsi + A.iCP + 2 * NN * j + NN};
    };
    bool fail = ncp > A.cp_max || s - 1 > A.sg_max || N > A.Ncap;
    int64_t bp_sum = 0;
    int bp_max = 0;
    // forward: leaves into W[(N+1) & 1] and checkpoint 0
    if (!fail) {
        const LevelRef L = W[(N + 1) & 1];
        for (int c = tid; c <= N + 1; c += WG) {
            const double S = Stab[2 * c];
            double *r = L.rec + 4 * (int64_t)c;
            r[0] = -((1.0 + md.k) * S); r[1] = 0.0; r[2] = 0.0; r[3] = -((1.0 - md.k) * S);
            L.off[c] = 4 * c;
            L.cnt[c] = 1;
        }
        if (tid == 0) cp_base[0] = 0;
        __syncthreads();
        copy_level(L, cp_level(0), N + 2, 4 * NN);
        if (tid == 0) cp_base[1] = 4 * NN;
        __syncthreads();
    }
    for (int t = N; t >= 1 && !fail; t--) {
        const int64_t nn = adj_fwd_level<SIDE>(A, md, t, Stab, W[(t + 1) & 1], W[t & 1], A.lwn, lane, big, &bp_sum,
                                               &bp_max, sh, sbig, srun, sflag);
        if (nn < 0) { fail = true; break; }
        if ((N + 1 - t) % s == 0) {
            const int j = (N + 1 - t) / s;
            if (cp_base[j] + nn > A.cp_nums) { fail = true; break; }
            copy_level(W[t & 1], cp_level(j), t + 1, nn);
            if (tid == 0 && j + 1 < A.cp_max + 1) cp_base[j + 1] = cp_base[j] + nn;
            __syncthreads();
        }
    }
    // reverse, root side first
    GAcc g{0.0, 0.0, 0.0, 0.0};
    double price = 0.0;
    int cur = 0;
    int lo = 0;
    for (int jj = ncp - 1; jj >= 0 && !fail; jj--) {
        const int hi = N + 1 - jj * s;
        // levels lo+1 .. hi-1 recomputed from checkpoint jj into the segment
        // region: level t at slot hi-1-t
        int64_t seg_used = 0;
        const auto seg_level = [&](int t, int64_t base) {
            const int slot = hi - 1 - t;
            return LevelRef{ws + A.oSG + base, wsi + A.iSG + 2 * NN * slot, wsi + A.iSG + 2 * NN * slot + NN};
        };
        LevelRef up = cp_level(jj);
        for (int t = hi - 1; t >= lo + 1; t--) {
            const LevelRef dst = seg_level(t, seg_used);
            int64_t dsum = 0;
            int dmax = 0;
            const int64_t nn = adj_fwd_level<SIDE>(A, md, t, Stab, up, dst, A.sg_nums - seg_used, lane, big, &dsum,
                                                   &dmax, sh, sbig, srun, sflag);
            if (nn < 0) { fail = true; break; }
            if (tid == 0) sg_base[hi - 1 - t] = seg_used;
            seg_used += nn;
            up = dst;
        }
        __syncthreads();
        if (fail) break;
        const auto level_at = [&](int t) {
            if (t == hi) return cp_level(jj);
            if (t == lo) return cp_level(jj + 1);
            const int slot = hi - 1 - t;
            return seg_level(t, sg_base[slot]);
        };
        for (int t = lo; t <= hi - 1; t++) {
            const LevelRef Lc = level_at(t + 1);
            const LevelRef Lt = t >= 1 ? level_at(t) : Lc;
            // numbers of level t+1: the last column's record ends the level
            // only when records are in column order, so sum the sizes
            int64_t nn = 0;
            for (int c = tid; c <= t + 1; c += WG) {
                const int64_t e = Lc.off[c] + 3 * (int64_t)Lc.cnt[c] + 1;
                nn = e > nn ? e : nn;
            }
            int64_t tmp;
            {
                // maximum over the workgroup
                for (int o = 32; o > 0; o >>= 1) {
                    const int64_t y = __shfl_down(nn, o, 64);
                    nn = y > nn ? y : nn;
                }
                if ((tid & 63) == 0) sh[tid >> 6] = nn;
                __syncthreads();
                tmp = 0;
                for (int q = 0; q < NWAVE; q++) tmp = sh[q] > tmp ? sh[q] : tmp;
                __syncthreads();
            }
            nn = tmp;
            if (nn > A.lwn) { fail = true; break; }
            double *Anxt = Abuf[cur ^ 1];
            if (!adj_rev_level<SIDE>(A, md, t, Stab, Sfac, Lt, Lc, nn, Abuf[cur], Anxt, lane, big, g, &price, sh, sbig,
                                     sflag)) {
                fail = true;
                break;
            }
            if (t == 0 && tid == 0) {
                // breakpoints of z_0 (the forward pass stopped at level 1)
                const View<double> Zd = level_view(Lc, 0), Zu = level_view(Lc, 1);
                const double S0 = Stab[N + 1];
                double xi, ze;
                payoff(md, in, S0, xi, ze);
                Arr<double> Z;
                const double kt0 = (md.flags & F_COST_AT_T0) ? md.k : 0.0;
                const bool ex0 = !((md.flags & F_EUROPEAN) && N > 0);
                const int m0 = node_update<SIDE, double>(Zu, Zd, S0, kt0, md.rho, xi, ze, ex0, big.fwd, 1, big.fcp, &Z);
                if (m0 < 0) *sflag = 1;
                else {
                    const int bp = (m0 == 1 && Z.S(0) == Z.S(1)) ? 0 : m0;
                    bp_sum += bp;
                    bp_max = bp > bp_max ? bp : bp_max;
                }
            }
            __syncthreads();
            if (*sflag) { fail = true; break; }
            cur ^= 1;
        }
        lo = hi;
    }
    if (!fail) {
        // the leaves: [-(1+k) S, 0, 0, -(1-k) S] per column
        const double *Al = Abuf[cur];
        for (int c = tid; c <= N + 1; c += WG) {
            const double S = Stab[2 * c];
            const double a0 = Al[4 * (int64_t)c], a1 = Al[4 * (int64_t)c + 3];
            const double gS = -(1.0 + md.k) * a0 - (1.0 - md.k) * a1;
            const int j = 2 * c - (N + 1);
            g.S0 += gS * Sfac[j + N + 1];
            g.sig += gS * (S * (double)j * md.sq);
            g.k += -S * a0 + S * a1;
        }
    }
    // workgroup sums in a fixed order
    __shared__ double s_g[NWAVE][4];
    __shared__ int64_t s_bp[NWAVE];
    __shared__ int s_bm[NWAVE];
    double v[4] = {g.S0, g.sig, g.R, g.k};
    int64_t bs = bp_sum;
    int bm = bp_max;
    for (int o = 32; o > 0; o >>= 1) {
        for (int q = 0; q < 4; q++) v[q] += __shfl_down(v[q], o, 64);
        bs += __shfl_down(bs, o, 64);
        const int y = __shfl_down(bm, o, 64);
        bm = y > bm ? y : bm;
    }
    __syncthreads();
    if ((tid & 63) == 0) {
        for (int q = 0; q < 4; q++) s_g[tid >> 6][q] = v[q];
        s_bp[tid >> 6] = bs;
        s_bm[tid >> 6] = bm;
    }
    __syncthreads();
    // the root step (column 0) ran on thread 0, as a small node or as wave
    // 0's large node: the price is in its register
    if (tid == 0) {
        double tg[4] = {0, 0, 0, 0};
        int64_t tb = 0;
        int tm = 0;
        for (int q = 0; q < NWAVE; q++) {
            for (int r = 0; r < 4; r++) tg[r] += s_g[q][r];
            tb += s_bp[q];
            tm = s_bm[q] > tm ? s_bm[q] : tm;
        }
        bt_result &o = A.out[opt];
        bt_grad4 &gg = SIDE == 0 ? A.grad[opt].ask : A.grad[opt].bid;
        if (fail) {
            atomicMin(&o.status, BT_EOVERFLOW);
        } else {
            if (SIDE == 0) { o.ask = price; o.bp_total_ask = tb; o.bp_max_ask = tm; }
            else { o.bid = -price; o.bp_total_bid = tb; o.bp_max_bid = tm; }
            gg.dS0 = tg[0]; gg.dsigma = tg[1]; gg.dR = tg[2]; gg.dk = tg[3];
        }
    }
    __syncthreads();
}

template <int SIDE>
__global__ __launch_bounds__(WG) void bt_adjoint_kernel(AdjArgs A)
{
    __shared__ int64_t sh[NWAVE];
    __shared__ int sbig[WG];
    __shared__ int64_t srun;
    __shared__ int sflag;
    __shared__ int s_q;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(A.queue + SIDE, 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= *A.count) break;
        adjoint_tree<SIDE>(A, A.order[q], sh, sbig, &srun, &sflag);
    }
}

// The exercise maps of options whose pricing failed are set to 0xff (one
// workgroup per option at a time).
__global__ void bt_exmap_fail_kernel(KArgs A)
{
    for (int64_t k = blockIdx.x; k < A.n_opts; k += gridDim.x) {
        if (A.out[k].status == BT_OK) continue;
        for (int64_t q = A.exoff[k] + threadIdx.x; q < A.exoff[k + 1]; q += blockDim.x) A.exmap[q] = 0xff;
    }
}

// Options whose pricing failed (status other than BT_OK: invalid, or a
// tree that outgrew its buffers on either side) get no partial result: NaN
// prices and Greeks, zero breakpoint counts.
__global__ void bt_finalize_kernel(KArgs A)
{
    const double nan = __builtin_nan("");
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.n_opts; k += (int64_t)gridDim.x * blockDim.x) {
        bt_result &o = A.out[k];
        if (o.status == BT_OK) continue;
        o.ask = nan; o.bid = nan; o.price0 = nan;
        o.bp_total_ask = 0; o.bp_total_bid = 0;
        o.bp_max_ask = 0; o.bp_max_bid = 0;
        if (A.grad) {
            bt_grad g;
            g.ask.dS0 = g.ask.dsigma = g.ask.dR = g.ask.dk = nan;
            g.bid = g.ask;
            A.grad[k] = g;
        }
        if (A.hedge) {
            bt_hedge h;
            h.ask_lo = h.ask_hi = h.bid_lo = h.bid_hi = nan;
            A.hedge[k] = h;
        }
    }
}

// ---------------------------------------------------------------------------
// Device planner of a batch whose options are in device memory
// (bt_price_batch): tree constants, the order of the tree sides and the band
// task lists, built on the GPU in the same order a book builds them on the
// host.  Every buffer is laid out for the batch's largest N, so nothing here
// depends on the host seeing the options.
// ---------------------------------------------------------------------------
struct PlanArgs {
    const bt_params *params;
    int n, max_N;
    Model *models;
    int2 *keys;          // per option: (N, or -1 when invalid; growth bits)
    int *order;          // [3][n]: buyer, seller and zero-cost orders (position -> option)
    int *count;          // valid options
    Item *items;         // [2n]: buyer tree sides at [0, n), seller tree sides at [n, 2n)
    Task *tasks;
    int *task_lo, *task_hi;
    int nbands_max, band, block_cols, lf, nt;
    int64_t lstride;     // doubles of band buffers per tree side
    int64_t istride;     // ints of offsets and counts per tree side
};

// Bits of the tree sides whose nodes grow large: 1 = the buyer of anything
// but a delivered put with costs, 2 = the seller of a cash-settled payoff
// with costs (the order a book uses puts them first in each party's task
// list).
BTHD int growth_bits(const Model &m)
{
    if (!m.valid || !(m.k > 0.0)) return 0;
    return (m.payoff != PAY_PUT ? 1 : 0) | (m.payoff >= PAY_BULL ? 2 : 0);
}

// Upper bound on the column blocks of one tree side in launch L: every tree
// side ends in the last launch, so its band in launch L starts at most
// (nbands - L) * band - 1 levels above the root.
BTHD int launch_blocks(int L, int nbands_max, int band, int block_cols)
{
    return ((nbands_max - L - 1) * band + 1 + block_cols - 1) / block_cols;
}

__global__ void bt_derive_kernel(PlanArgs P)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *P.count = 0;
    if (i >= P.n) return;
    Model m;
    const bool ok = derive_model(P.params[i], P.max_N, m);
    P.models[i] = m;
    P.keys[i] = make_int2(ok ? m.N : -1, growth_bits(m));
}

// Position of every valid option in the three orders, by counting the
// options that precede it: longer trees first, ties by index (zero-cost
// order); within a party the growing tree sides first, then the same.
__global__ __launch_bounds__(WG) void bt_rank_kernel(PlanArgs P)
{
    __shared__ int2 sk[WG];
    const int i = blockIdx.x * WG + threadIdx.x;
    const int2 ki = i < P.n ? P.keys[i] : make_int2(-1, 0);
    int pb = 0, ps = 0, pz = 0;
    for (int j0 = 0; j0 < P.n; j0 += WG) {
        __syncthreads();
        sk[threadIdx.x] = j0 + (int)threadIdx.x < P.n ? P.keys[j0 + threadIdx.x] : make_int2(-1, 0);
        __syncthreads();
        if (ki.x < 0) continue;
        const int jn = min(WG, P.n - j0);
        for (int jj = 0; jj < jn; jj++) {
            const int2 kj = sk[jj];
            if (kj.x < 0) continue;
            const bool first = kj.x > ki.x || (kj.x == ki.x && j0 + jj < i);
            const int gbj = kj.y & 1, gbi = ki.y & 1, gsj = (kj.y >> 1) & 1, gsi = (ki.y >> 1) & 1;
            pz += first;
            pb += gbj > gbi || (gbj == gbi && first);
            ps += gsj > gsi || (gsj == gsi && first);
        }
    }
    if (ki.x >= 0) {
        P.order[pb] = i;
        P.order[P.n + ps] = i;
        P.order[2 * P.n + pz] = i;
        atomicAdd(P.count, 1);
    }
}

// Tree side q: party slot q / n (0 buyer, 1 seller), position q % n.
__global__ void bt_items_kernel(PlanArgs P)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 2 * P.n) return;
    const int slot = q / P.n, pos = q - slot * P.n;
    Item it;
    it.side = slot == 0 ? 1 : 0;
    it.lbuf = (int64_t)q * P.lstride;
    it.ibuf = (int64_t)q * P.istride;
    it.ctr = (int64_t)q * (P.nbands_max + 1);
    if (pos < *P.count) {
        it.opt = P.order[slot * P.n + pos];
        it.N = P.models[it.opt].N;
        it.nbands = (it.N + P.band) / P.band;
        it.lcap = (((int64_t)P.lf * (it.N + 2) * 3 + (it.N + 2)) * P.nt + 31) & ~(int64_t)31;
    } else {
        it.opt = -1;
        it.N = 0;
        it.nbands = 0;
        it.lcap = 0;
    }
    P.items[q] = it;
}

// Task list of launch L (blockIdx.x), party blockIdx.y (0 seller, 1 buyer):
// the column blocks of every tree side of that party that launch L runs, in
// the party's order, in a region sized by launch_blocks.
__global__ __launch_bounds__(WG) void bt_tasks_kernel(PlanArgs P)
{
    __shared__ int64_t sh[NWAVE];
    const int L = blockIdx.x, side = blockIdx.y, slot = side == 1 ? 0 : 1;
    int64_t base = 0;
    for (int l = 0; l < L; l++) base += 2 * (int64_t)launch_blocks(l, P.nbands_max, P.band, P.block_cols);
    base += side * (int64_t)launch_blocks(L, P.nbands_max, P.band, P.block_cols);
    base *= P.n;
    const int cnt = *P.count;
    int64_t run = 0;
    for (int p0 = 0; p0 < cnt; p0 += WG) {
        const int pos = p0 + threadIdx.x;
        const int q = slot * P.n + pos;
        int nb = 0;
        if (pos < cnt) {
            const Item I = P.items[q];
            const int r = L - (P.nbands_max - I.nbands);
            if (r >= 0) {
                const int t_top = I.N - r * P.band;
                const int t_bot = t_top - P.band + 1 > 0 ? t_top - P.band + 1 : 0;
                nb = (t_bot + 1 + P.block_cols - 1) / P.block_cols;
            }
        }
        int64_t tot;
        const int64_t ex = block_scan(nb, &tot, sh);
        for (int b = 0; b < nb; b++) P.tasks[base + run + ex + b] = Task{q, b};
        run += tot;
    }
    if (threadIdx.x == 0) {
        P.task_lo[2 * L + side] = (int)base;
        P.task_hi[2 * L + side] = (int)(base + run);
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
thread_local int g_last_hip = 0;
// What bt_price keeps between calls on a thread (freed by bt_shutdown).
thread_local bt_result *t_price_res = nullptr;
thread_local bt_book *t_price_book = nullptr;
thread_local int t_price_N = -1;

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
bool derive(const bt_params &p, Model &m) { return derive_model(p, BT_MAX_N, m); }

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct bt_book {
    int device = 0;
    int n = 0, n_max = 0, n_items = 0, nbands_max = 0;
    int64_t nodes = 0, n_fill = 0;
    int grid = 0, grid_p0 = 0;
    bool greeks = false;           // buffers sized for dual numbers
    std::vector<int> ntasks;       // per (band, side)
    Model *d_models = nullptr;
    Item *d_items = nullptr;
    Task *d_tasks = nullptr;
    int *d_task_off = nullptr;
    int *d_ints = nullptr;         // band counters, failure flags, price0 queue and schedule
    unsigned long long *d_fill = nullptr;
    double *d_lvl = nullptr;
    int *d_lvli = nullptr;
    double *d_ws = nullptr;
    int *d_wsi = nullptr;
    double *d_arena = nullptr;
    unsigned long long *d_arena_ctr = nullptr;
    double *d_wsp = nullptr;
    // the seller's bands and the zero-cost recursion run on streams of
    // their own, forked from and joined to the caller's stream
    hipStream_t s_ask = nullptr, s_p0 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_ask = nullptr, ev_p0 = nullptr;
    KArgs args{};
    bool timing = false;
    std::vector<hipEvent_t> events;  // NEV per timed call
    // BT_TUNE_GRAPH: the launch sequence captured once per (output buffers,
    // number type) on an internal stream, replayed on the caller's stream
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bt_result *g_out = nullptr;
    bt_grad *g_grad = nullptr;
    int g_nt = 0;
    std::vector<bt_params> params;   // host copy, for re-pricing on overflow
    bt_tune tune{};
    // a batch workspace (bt_price_batch): planned on the device for up to
    // cap_n options of up to cap_N steps each
    bool device_plan = false;
    bool carved = false;              // buffers carved from a caller's region: not freed here
    int cap_n = 0, cap_N = 0;
    int2 *d_keys = nullptr;
    int *d_order = nullptr;
    int *d_plan_ints = nullptr;       // valid count, task bounds
    PlanArgs plan{};
    int64_t *d_exoff = nullptr;       // exercise-map offsets (first bt_book_price_exercise)
};

namespace {

void book_free(bt_book *b)
{
    if (!b) return;
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_ask) (void)hipEventDestroy(b->ev_ask);
    if (b->ev_p0) (void)hipEventDestroy(b->ev_p0);
    if (b->s_ask) (void)hipStreamDestroy(b->s_ask);
    if (b->s_p0) (void)hipStreamDestroy(b->s_p0);
    b->ev_fork = b->ev_ask = b->ev_p0 = nullptr;
    b->s_ask = b->s_p0 = nullptr;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->cap_stream = nullptr;
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    b->events.clear();
    void *ptrs[] = {b->d_models, b->d_items, b->d_tasks, b->d_task_off, b->d_ints,
                    b->d_fill, b->d_lvl, b->d_lvli, b->d_ws, b->d_wsi, b->d_arena, b->d_arena_ctr, b->d_wsp,
                    b->d_keys, b->d_order, b->d_plan_ints};
    for (void *p : ptrs)
        if (p && !b->carved) (void)hipFree(p);
    if (b->d_exoff) (void)hipFree(b->d_exoff);
    b->d_exoff = nullptr;
    b->d_keys = nullptr; b->d_order = nullptr; b->d_plan_ints = nullptr;
    b->d_models = nullptr; b->d_items = nullptr; b->d_tasks = nullptr; b->d_task_off = nullptr;
    b->d_ints = nullptr; b->d_fill = nullptr; b->d_lvl = nullptr; b->d_lvli = nullptr;
    b->d_ws = nullptr; b->d_wsi = nullptr; b->d_arena = nullptr; b->d_arena_ctr = nullptr; b->d_wsp = nullptr;
}

template <typename T>
int dalloc(T **p, size_t count)
{
    if (hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return BT_ENOMEM;
    }
    return BT_OK;
}

// Doubles of arena that one party of a book may need: the temporaries of
// the nodes too big for a wave's pool slice (`slice` doubles).  The buyer of
// a call or a bull spread with costs grows nodes of up to about 2N to 2.7N
// breakpoints (13512 at N = 5000, 16175 at N = 8129), so a node's two
// children hold up to about 5N; a bull spread's seller stays near N; puts
// stay at a few points.  Tree sides are aligned at the root, so their
// largest nodes meet in the same launches; near the root a tree side is one
// task, so at most `conc` of them (the resident workgroups) hold big nodes
// at once: the largest `conc` count three big nodes per level, each taking
// up to twice its need (a wave takes 1.25 times its first need and keeps the
// chunk for the whole launch, doubling it when a later node outgrows it).  The estimate only sizes the allocation: an option
// whose nodes outgrow it is reported BT_EOVERFLOW, and
// bt_book_resolve_overflow re-prices it.
int64_t arena_estimate(const std::vector<Model> &models, const std::vector<Item> &items, int side,
                       int64_t slice, int64_t nt, int conc)
{
    std::vector<int64_t> needs;
    for (const Item &it : items) {
        const Model &m = models[it.opt];
        if (it.side != side || !(m.k > 0)) continue;
        int64_t M = 0;
        if (side == 1 && m.payoff != BT_PUT) M = 5 * (int64_t)it.N;
        if (side == 0 && m.payoff >= BT_BULL) M = it.N;
        const int64_t need = (64 * M + 4096) * nt;   // as big_need on the device
        if (need > slice) needs.push_back(need);
    }
    std::sort(needs.begin(), needs.end(), std::greater<int64_t>());
    int64_t est = 0;
    for (size_t i = 0; i < needs.size() && i < (size_t)conc; i++) {
        est += 3 * 2 * needs[i];
        if (est >= MAX_ARENA_DOUBLES) return MAX_ARENA_DOUBLES;
    }
    return est;
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
    const int lf = (tune && tune->level_factor > 0) ? tune->level_factor : DEFAULT_LEVEL_FACTOR;
    const bool greeks = tune && (tune->flags & BT_TUNE_GREEKS);
    const int64_t nt = greeks ? (int64_t)(sizeof(D4) / sizeof(double)) : 1;  // doubles per number
    const int wpc = (tune && tune->wgs_per_cu > 0) ? tune->wgs_per_cu : 2;
    if (tune && tune->band_levels != 0 && (tune->band_levels < MIN_BAND || tune->band_levels > BAND)) return BT_EINVAL;
    const int band = (tune && tune->band_levels > 0) ? tune->band_levels : BAND;
    const int block_cols = WG - band;
    const int64_t pool_pts = (tune && tune->pool_points > 0) ? (int64_t)tune->pool_points
                                                             : (greeks ? DEFAULT_POOL_POINTS / 4 : DEFAULT_POOL_POINTS);
    const int64_t pool = pool_pts * 4 * nt;
    const int64_t arena_floor = std::max<int64_t>(DEFAULT_ARENA_DOUBLES * nt, 64 * pool);

    // tree sides, buyer first (the longer recursion).  Within a party the
    // sides whose nodes grow large (costly call and bull-spread buyers,
    // costly bull-spread sellers) come first, then the longest trees: a
    // launch's task list follows this order, so its slowest tasks start
    // first
    std::vector<int> order;
    for (int i = 0; i < n; i++)
        if (models[i].valid) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return models[x].N > models[y].N; });
    const auto grows = [&](int i, int side) {
        const Model &m = models[i];
        return m.k > 0 && (side == 1 ? m.payoff != BT_PUT : m.payoff >= BT_BULL);
    };
    std::vector<Item> items;
    int64_t lbuf = 0, ibuf = 0, ctr = 0;
    int nbands_max = 0;
    for (int side = 1; side >= 0; side--) {
        std::vector<int> so(order);
        std::stable_sort(so.begin(), so.end(), [&](int x, int y) {
            const bool gx = grows(x, side), gy = grows(y, side);
            return gx != gy ? gx : models[x].N > models[y].N;
        });
        for (int i : so) {
            Item it;
            it.opt = i; it.side = side; it.N = models[i].N;
            it.nbands = (it.N + 1 + band - 1) / band;
            it.lcap = round_up(((int64_t)lf * (it.N + 2) * 3 + (it.N + 2)) * nt, 32);
            it.lbuf = lbuf; lbuf += 2 * it.lcap;
            it.ibuf = ibuf; ibuf += round_up(4 * (int64_t)(it.N + 2), 32);
            it.ctr = ctr; ctr += it.nbands + 1;
            nbands_max = std::max(nbands_max, it.nbands);
            items.push_back(it);
        }
    }
    // band tasks, grouped by (launch, side); launch L runs band
    // L - (nbands_max - nbands) of each tree side, so that all end together
    std::vector<Task> tasks;
    std::vector<int> task_off(2 * (size_t)nbands_max + 1, 0);
    std::vector<int> ntasks(2 * (size_t)nbands_max, 0);
    for (int L = 0; L < nbands_max; L++) {
        for (int side = 0; side < 2; side++) {
            task_off[2 * L + side] = (int)tasks.size();
            for (int q = 0; q < (int)items.size(); q++) {
                const Item &it = items[q];
                const int r = L - (nbands_max - it.nbands);
                if (it.side != side || r < 0) continue;
                const int t_top = it.N - r * band;
                const int t_bot = std::max(t_top - band + 1, 0);
                const int nb = (t_bot + 1 + block_cols - 1) / block_cols;
                for (int bk = 0; bk < nb; bk++) tasks.push_back(Task{q, bk});
            }
            ntasks[2 * L + side] = (int)tasks.size() - task_off[2 * L + side];
        }
    }
    task_off[2 * (size_t)nbands_max] = (int)tasks.size();
    std::vector<int> p0(order);

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    int max_tasks = 1;
    for (int v : ntasks) max_tasks = std::max(max_tasks, v);
    const int resident = prop.multiProcessorCount * wpc;
    const int grid = std::max(1, std::min(max_tasks, resident));
    const int grid_p0 = std::max(1, std::min((int)p0.size(), resident));
    const int ws_wgs = grid;
    // each party's arena: its estimate, at least the floor, and beyond the
    // floor at most an eighth of the device's free memory
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = 0;
    }
    int64_t arena[2];
    for (int side = 0; side < 2; side++) {
        const int64_t e = std::min<int64_t>(arena_estimate(models, items, side, pool / NWAVE, nt, grid),
                                            (int64_t)(free_b / 8 / sizeof(double)));
        arena[side] = round_up(std::max(arena_floor, e), 32);
    }

    KArgs a{};
    // a private level holds the records of WG + 1 columns: lf breakpoints per
    // node on average, and never fewer than MIN_PRIVATE_POINTS (scaled up
    // with lf) in all, since a few nodes of a level can hold most of its
    // breakpoints.  The buyer of a call or a bull spread with costs reaches
    // about 2N breakpoints per node (16175 at N = 8129) with several such
    // nodes in a block, so such a book's levels get 16N points.
    int64_t ppts = std::max((int64_t)lf * (WG + 1), MIN_PRIVATE_POINTS * std::max(1, lf / DEFAULT_LEVEL_FACTOR));
    for (const Item &it : items)
        if (it.side == 1 && models[it.opt].k > 0 && models[it.opt].payoff != BT_PUT)
            ppts = std::max(ppts, 16 * (int64_t)it.N);
    const int64_t pcap = round_up(ppts * 3 * nt + (WG + 1) * nt, 32);
    // offsets into a band buffer or a private level are int
    if ((int64_t)lf * (n_max + 2) * 3 + (n_max + 2) > INT32_MAX || ppts * 3 + (WG + 1) > INT32_MAX) return BT_EINVAL;
    const Caps sc = small_caps();
    a.oStab = 0;
    const int64_t stab_n = std::max<int64_t>((2 * (int64_t)WG + BAND + 8) * nt, 2 * (int64_t)n_max + 3);
    a.oP0 = round_up(stab_n, 32);
    a.oP1 = a.oP0 + pcap;
    a.oSmall = a.oP1 + pcap;
    a.oPool = a.oSmall + round_up(sc.total * WG * nt, 32);
    a.ws_doubles = a.oPool + round_up(std::max<int64_t>(pool, 2 * (int64_t)n_max + 4), 32);
    a.wsi_ints = round_up(4 * (int64_t)(WG + 1), 64);
    a.ws_side = a.ws_doubles * ws_wgs;
    a.wsi_side = a.wsi_ints * ws_wgs;
    a.p0_stab = round_up(2 * (int64_t)n_max + 3, 32);
    a.p0_doubles = a.p0_stab + round_up(2 * (int64_t)n_max + 2, 32);
    a.pcap = pcap;
    a.pool = pool;
    a.n_opts = n;
    a.n_items = (int)items.size();
    a.nbands_max = nbands_max;
    a.band = band;

    b->use_graph = tune && (tune->flags & BT_TUNE_GRAPH);
    b->timing = tune && (tune->flags & BT_TUNE_TIMING) && !b->use_graph;
    b->greeks = greeks;
    b->params.assign(h, h + n);
    if (tune) b->tune = *tune;
    b->device = dev;
    b->n = n; b->n_max = n_max; b->nodes = nodes; b->n_items = (int)items.size();
    b->nbands_max = nbands_max;
    b->n_fill = ctr;
    b->grid = grid; b->grid_p0 = grid_p0;
    b->ntasks = ntasks;

    const int64_t nints = 2 * (int64_t)nbands_max + (int64_t)items.size() + 64 + (int64_t)p0.size() + 1;
    int rc = BT_OK;
    if ((rc = dalloc(&b->d_models, n)) || (rc = dalloc(&b->d_items, items.size())) ||
        (rc = dalloc(&b->d_tasks, tasks.size())) || (rc = dalloc(&b->d_task_off, task_off.size())) ||
        (rc = dalloc(&b->d_ints, nints)) || (rc = dalloc(&b->d_fill, ctr)) ||
        (rc = dalloc(&b->d_lvl, lbuf)) || (rc = dalloc(&b->d_lvli, ibuf)) ||
        (rc = dalloc(&b->d_ws, 2 * a.ws_side)) || (rc = dalloc(&b->d_wsi, 2 * a.wsi_side)) ||
        (rc = dalloc(&b->d_wsp, a.p0_doubles * grid_p0)) ||
        (rc = dalloc(&b->d_arena, arena[0] + arena[1])) || (rc = dalloc(&b->d_arena_ctr, 2 * (size_t)nbands_max))) {
        book_free(b);
        return rc;
    }
    HIPCHK(hipMemcpy(b->d_models, models.data(), sizeof(Model) * n, hipMemcpyHostToDevice));
    if (!items.empty()) HIPCHK(hipMemcpy(b->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    if (!tasks.empty()) HIPCHK(hipMemcpy(b->d_tasks, tasks.data(), sizeof(Task) * tasks.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_task_off, task_off.data(), sizeof(int) * task_off.size(), hipMemcpyHostToDevice));
    int *band_ctr = b->d_ints;
    int *failed = band_ctr + 2 * (int64_t)nbands_max;
    int *p0q = failed + items.size();
    int *p0s = p0q + 64;
    int *p0n = p0s + p0.size();
    if (!p0.empty()) HIPCHK(hipMemcpy(p0s, p0.data(), sizeof(int) * p0.size(), hipMemcpyHostToDevice));
    const int n_p0 = (int)p0.size();
    HIPCHK(hipMemcpy(p0n, &n_p0, sizeof(int), hipMemcpyHostToDevice));
    a.models = b->d_models;
    a.items = b->d_items;
    a.tasks = b->d_tasks;
    a.task_lo = b->d_task_off;
    a.task_hi = b->d_task_off + 1;
    a.band_ctr = band_ctr;
    a.fill = b->d_fill;
    a.failed = failed;
    a.lvl = b->d_lvl;
    a.lvli = b->d_lvli;
    a.ws = b->d_ws;
    a.wsi = b->d_wsi;
    a.wsp = b->d_wsp;
    a.p0_queue = p0q;
    a.p0_sched = p0s;
    a.p0_count = p0n;
    a.arena = b->d_arena;
    a.arena_cap[0] = arena[0];
    a.arena_cap[1] = arena[1];
    a.arena_base[0] = 0;
    a.arena_base[1] = arena[0];
    a.arena_ctr = b->d_arena_ctr;
    b->args = a;
    HIPCHK(hipStreamCreateWithFlags(&b->s_ask, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&b->s_p0, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_ask, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_p0, hipEventDisableTiming));
    return BT_OK;
}

// Carves device buffers out of one region (a caller-provided scratch area)
// or allocates each with hipMalloc.
struct Carver {
    char *base = nullptr;     // nullptr: hipMalloc each buffer
    size_t cap = 0, used = 0;
    template <typename T>
    int take(T **p, size_t count)
    {
        const size_t bytes = (sizeof(T) * std::max<size_t>(count, 1) + 255) & ~(size_t)255;
        if (!base) return dalloc(p, count);
        if (used + bytes > cap) return BT_ENOMEM;
        *p = (T *)(base + used);
        used += bytes;
        return BT_OK;
    }
};

// Tuning of a batch workspace with the library's defaults filled in.
bt_tune batch_tune(const bt_tune *tune, bool greeks)
{
    bt_tune t{};
    if (tune) t = *tune;
    t.flags = greeks ? BT_TUNE_GREEKS : 0;
    if (t.wgs_per_cu <= 0) t.wgs_per_cu = 1;   // the LDS of one band workgroup fills a CU
    if (t.level_factor <= 0) t.level_factor = DEFAULT_LEVEL_FACTOR;
    if (t.pool_points <= 0) t.pool_points = (int32_t)(greeks ? DEFAULT_POOL_POINTS / 4 : DEFAULT_POOL_POINTS);
    if (t.band_levels == 0) t.band_levels = BAND;
    return t;
}

// Workspace of a batch planned on the device: every buffer sized for cap_n
// options of up to cap_N steps each, as if every option were the buyer of a
// costly call (the largest nodes): two band buffers per tree side, private
// levels of 16 cap_N points, and each party's arena estimated like a book's
// for min(cap_n, resident workgroups) such tree sides, between the book's
// floor and arena_cap doubles.  The buffers come from `carve` (hipMalloc, or a
// caller's region).  `grid_cap` (0: none) bounds the persistent workgroups.
int batch_build(bt_book *b, int cap_n, int cap_N, const bt_tune &t, int grid_cap, int64_t arena_cap, Carver &cv,
                int64_t min_private = MIN_PRIVATE_POINTS, bool streams = true)
{
    const bool greeks = (t.flags & BT_TUNE_GREEKS) != 0;
    const int64_t nt = greeks ? (int64_t)(sizeof(D4) / sizeof(double)) : 1;
    if (t.band_levels < MIN_BAND || t.band_levels > BAND || cap_n < 1 || cap_N < 1 || cap_N > BT_MAX_N) return BT_EINVAL;
    const int band = t.band_levels, block_cols = WG - band, lf = t.level_factor;
    const int nbands_max = (cap_N + band) / band;
    const int64_t pool = (int64_t)t.pool_points * 4 * nt;
    const int64_t arena_floor = std::min(std::max<int64_t>(DEFAULT_ARENA_DOUBLES * nt, 64 * pool), arena_cap);
    int64_t ppts = std::max({(int64_t)lf * (WG + 1), min_private * std::max(1, lf / DEFAULT_LEVEL_FACTOR),
                             16 * (int64_t)cap_N});
    if ((int64_t)lf * (cap_N + 2) * 3 + (cap_N + 2) > INT32_MAX || ppts * 3 + (WG + 1) > INT32_MAX) return BT_EINVAL;
    // task capacity: cap_n tree sides per party, launch_blocks each
    int64_t task_cap = 0;
    for (int L = 0; L < nbands_max; L++) task_cap += 2 * (int64_t)launch_blocks(L, nbands_max, band, block_cols);
    task_cap *= cap_n;
    if (task_cap > INT32_MAX) return BT_EINVAL;

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    int grid = prop.multiProcessorCount * t.wgs_per_cu;
    if (grid_cap > 0) grid = std::min(grid, grid_cap);
    const int grid_p0 = std::max(1, std::min(cap_n, grid));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = 0;
    }
    int64_t arena[2];
    for (int side = 0; side < 2; side++) {
        const int64_t M = side == 1 ? 5 * (int64_t)cap_N : cap_N;
        const int64_t need = (64 * M + 4096) * nt;
        const int64_t est = need > pool / NWAVE ? 3 * 2 * need * std::min(cap_n, grid) : 0;
        int64_t e = std::min({est, arena_cap, (int64_t)(free_b / 8 / sizeof(double))});
        arena[side] = round_up(std::max(arena_floor, e), 32);
    }

    KArgs a{};
    const int64_t lstride = 2 * round_up(((int64_t)lf * (cap_N + 2) * 3 + (cap_N + 2)) * nt, 32);
    const int64_t istride = round_up(4 * (int64_t)(cap_N + 2), 32);
    const int64_t pcap = round_up(ppts * 3 * nt + (WG + 1) * nt, 32);
    const Caps sc = small_caps();
    a.oStab = 0;
    const int64_t stab_n = std::max<int64_t>((2 * (int64_t)WG + BAND + 8) * nt, 2 * (int64_t)cap_N + 3);
    a.oP0 = round_up(stab_n, 32);
    a.oP1 = a.oP0 + pcap;
    a.oSmall = a.oP1 + pcap;
    a.oPool = a.oSmall + round_up(sc.total * WG * nt, 32);
    a.ws_doubles = a.oPool + round_up(std::max<int64_t>(pool, 2 * (int64_t)cap_N + 4), 32);
    a.wsi_ints = round_up(4 * (int64_t)(WG + 1), 64);
    a.ws_side = a.ws_doubles * grid;
    a.wsi_side = a.wsi_ints * grid;
    a.p0_stab = round_up(2 * (int64_t)cap_N + 3, 32);
    a.p0_doubles = a.p0_stab + round_up(2 * (int64_t)cap_N + 2, 32);
    a.pcap = pcap;
    a.pool = pool;
    a.nbands_max = nbands_max;
    a.band = band;

    const int64_t n_items = 2 * (int64_t)cap_n;
    const int64_t n_fill = n_items * (nbands_max + 1);
    const int64_t nints = 2 * (int64_t)nbands_max + n_items + 64;
    int rc = BT_OK;
    if ((rc = cv.take(&b->d_models, cap_n)) || (rc = cv.take(&b->d_keys, cap_n)) ||
        (rc = cv.take(&b->d_order, 3 * (size_t)cap_n)) || (rc = cv.take(&b->d_plan_ints, 1 + 4 * (size_t)nbands_max)) ||
        (rc = cv.take(&b->d_items, n_items)) || (rc = cv.take(&b->d_tasks, task_cap)) ||
        (rc = cv.take(&b->d_ints, nints)) || (rc = cv.take(&b->d_fill, n_fill)) ||
        (rc = cv.take(&b->d_lvl, n_items * lstride)) || (rc = cv.take(&b->d_lvli, n_items * istride)) ||
        (rc = cv.take(&b->d_ws, 2 * a.ws_side)) || (rc = cv.take(&b->d_wsi, 2 * a.wsi_side)) ||
        (rc = cv.take(&b->d_wsp, a.p0_doubles * grid_p0)) ||
        (rc = cv.take(&b->d_arena, arena[0] + arena[1])) || (rc = cv.take(&b->d_arena_ctr, 2 * (size_t)nbands_max)))
        return rc;
    int *band_ctr = b->d_ints;
    int *failed = band_ctr + 2 * (int64_t)nbands_max;
    int *p0q = failed + n_items;
    int *count = b->d_plan_ints;
    int *task_lo = count + 1, *task_hi = task_lo + 2 * nbands_max;
    a.models = b->d_models;
    a.items = b->d_items;
    a.tasks = b->d_tasks;
    a.task_lo = task_lo;
    a.task_hi = task_hi;
    a.band_ctr = band_ctr;
    a.fill = b->d_fill;
    a.failed = failed;
    a.lvl = b->d_lvl;
    a.lvli = b->d_lvli;
    a.ws = b->d_ws;
    a.wsi = b->d_wsi;
    a.wsp = b->d_wsp;
    a.p0_queue = p0q;
    a.p0_count = count;
    a.arena = b->d_arena;
    a.arena_cap[0] = arena[0];
    a.arena_cap[1] = arena[1];
    a.arena_base[0] = 0;
    a.arena_base[1] = arena[0];
    a.arena_ctr = b->d_arena_ctr;
    b->args = a;

    PlanArgs &P = b->plan;
    P.models = b->d_models;
    P.keys = b->d_keys;
    P.order = b->d_order;
    P.count = count;
    P.items = b->d_items;
    P.tasks = b->d_tasks;
    P.task_lo = task_lo;
    P.task_hi = task_hi;
    P.nbands_max = nbands_max;
    P.band = band;
    P.block_cols = block_cols;
    P.lf = lf;
    P.nt = (int)nt;
    P.lstride = lstride;
    P.istride = istride;

    b->device_plan = true;
    b->cap_n = cap_n;
    b->cap_N = cap_N;
    b->greeks = greeks;
    b->tune = t;
    b->device = dev;
    b->n = cap_n; b->n_max = cap_N; b->n_items = (int)n_items;
    b->nbands_max = nbands_max;
    b->n_fill = n_fill;
    b->grid = grid; b->grid_p0 = grid_p0;
    if (!streams) return BT_OK;
    HIPCHK(hipStreamCreateWithFlags(&b->s_ask, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&b->s_p0, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_ask, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_p0, hipEventDisableTiming));
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

}  // extern "C"

namespace {

// Reset and level N+1 on the caller's stream, then three independent
// recursions: the buyer's bands there, the seller's bands and the zero-cost
// recursion on the book's own streams (forked from the caller's and joined
// back to it).  When the book times its calls, events bracket the groups:
// setup, buyer, seller, zero-cost (BT_NUM_KERNELS, kept per call as
// NEV events).
constexpr int NEV = 7;

template <typename T>
int launch_all(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream, const bt_params *d_params = nullptr,
               int n_call = 0, int max_N_call = 0, bt_hedge *d_hedge = nullptr, unsigned char *d_exmap = nullptr)
{
    hipStream_t s = (hipStream_t)stream;
    KArgs a = book->args;
    a.out = d_out;
    a.grad = d_grad;
    a.hedge = d_hedge;
    a.exmap = d_exmap;
    a.exoff = d_exmap ? book->d_exoff : nullptr;
    int64_t n_fill = book->n_fill;
    int n_opts = book->n;
    if (book->device_plan) {
        // plan on the device: constants, orders, tree sides, task lists
        PlanArgs P = book->plan;
        P.params = d_params;
        P.n = n_call;
        P.max_N = max_N_call;
        a.n_opts = n_call;
        a.n_items = 2 * n_call;
        a.p0_sched = book->d_order + 2 * (int64_t)n_call;
        n_fill = (int64_t)a.n_items * (book->nbands_max + 1);
        n_opts = n_call;
        const int g1 = (n_call + WG - 1) / WG, g2 = (2 * n_call + WG - 1) / WG;
        hipLaunchKernelGGL(bt_derive_kernel, dim3(g1), dim3(WG), 0, s, P);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(bt_rank_kernel, dim3(g1), dim3(WG), 0, s, P);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(bt_items_kernel, dim3(g2), dim3(WG), 0, s, P);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(bt_tasks_kernel, dim3(book->nbands_max, 2), dim3(WG), 0, s, P);
        HIPCHK(hipGetLastError());
    }
    hipEvent_t ev[NEV];
    if (book->timing) {
        for (int i = 0; i < NEV; i++) HIPCHK(hipEventCreate(&ev[i]));
        for (int i = 0; i < NEV; i++) book->events.push_back(ev[i]);
        HIPCHK(hipEventRecord(ev[0], s));
    }
    const int64_t nr = std::max<int64_t>({(int64_t)n_opts, 2 * (int64_t)book->nbands_max, n_fill,
                                          (int64_t)a.n_items, 1});
    const int rb = (int)std::min<int64_t>((nr + 255) / 256, 1024);
    hipLaunchKernelGGL(bt_reset_kernel, dim3(rb), dim3(256), 0, s, a, n_fill);
    HIPCHK(hipGetLastError());
    if (a.n_items > 0) {
        hipLaunchKernelGGL(bt_init_kernel<T>, dim3((book->n_max + 2 + 255) / 256, std::min(a.n_items, 65535)), dim3(256),
                           0, s, a);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[1], s));
    // a workspace without streams of its own runs the three recursions one
    // after the other on the caller's stream
    const bool fork = book->s_ask != nullptr;
    hipStream_t s_ask = fork ? book->s_ask : s, s_p0 = fork ? book->s_p0 : s;
    if (fork) {
        HIPCHK(hipEventRecord(book->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(s_ask, book->ev_fork, 0));
        HIPCHK(hipStreamWaitEvent(s_p0, book->ev_fork, 0));
    }
    // buyer
    // (a batch planned on the device runs every launch; its task counts are
    // on the device)
    const auto wgs = [&](int r, int side) {
        return book->device_plan ? book->grid : std::min(book->grid, book->ntasks[2 * r + side]);
    };
    // (with exercise maps: the kernels that also write them)
    for (int r = 0; r < book->nbands_max; r++) {
        if (wgs(r, 1) == 0) continue;
        if (d_exmap) hipLaunchKernelGGL((bt_band_kernel<1, double, true>), dim3(wgs(r, 1)), dim3(WG), 0, s, a, r);
        else hipLaunchKernelGGL((bt_band_kernel<1, T>), dim3(wgs(r, 1)), dim3(WG), 0, s, a, r);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[2], s));
    // seller
    if (book->timing) HIPCHK(hipEventRecord(ev[3], s_ask));
    for (int r = 0; r < book->nbands_max; r++) {
        if (wgs(r, 0) == 0) continue;
        if (d_exmap) hipLaunchKernelGGL((bt_band_kernel<0, double, true>), dim3(wgs(r, 0)), dim3(WG), 0, s_ask, a, r);
        else hipLaunchKernelGGL((bt_band_kernel<0, T>), dim3(wgs(r, 0)), dim3(WG), 0, s_ask, a, r);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[4], s_ask));
    // zero-cost recursion
    if (book->timing) HIPCHK(hipEventRecord(ev[5], s_p0));
    if (book->device_plan || book->n_items > 0) {
        hipLaunchKernelGGL(bt_price0_kernel, dim3(book->grid_p0), dim3(WG), 0, s_p0, a);
        HIPCHK(hipGetLastError());
    }
    if (book->timing) HIPCHK(hipEventRecord(ev[6], s_p0));
    if (fork) {
        HIPCHK(hipEventRecord(book->ev_ask, s_ask));
        HIPCHK(hipEventRecord(book->ev_p0, s_p0));
        HIPCHK(hipStreamWaitEvent(s, book->ev_ask, 0));
        HIPCHK(hipStreamWaitEvent(s, book->ev_p0, 0));
    }
    hipLaunchKernelGGL(bt_finalize_kernel, dim3((int)std::min<int64_t>((n_opts + 255) / 256, 1024)), dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
    if (d_exmap && n_opts > 0) {
        hipLaunchKernelGGL(bt_exmap_fail_kernel, dim3(std::min(n_opts, 1024)), dim3(256), 0, s, a);
        HIPCHK(hipGetLastError());
    }
    return BT_OK;
}

// The launch sequence directly, or as a replay of its captured graph.
template <typename T>
int launch(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream)
{
    if (!book->use_graph) return launch_all<T>(book, d_out, d_grad, stream);
    const int nt = (int)(sizeof(T) / sizeof(double));
    if (!book->gexec || book->g_out != d_out || book->g_grad != d_grad || book->g_nt != nt) {
        if (book->gexec) HIPCHK(hipGraphExecDestroy(book->gexec));
        if (book->graph) HIPCHK(hipGraphDestroy(book->graph));
        book->gexec = nullptr;
        book->graph = nullptr;
        if (!book->cap_stream) HIPCHK(hipStreamCreateWithFlags(&book->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(book->cap_stream, hipStreamCaptureModeThreadLocal));
        const int rc = launch_all<T>(book, d_out, d_grad, book->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(book->cap_stream, &g);
        if (rc != BT_OK) {
            if (e == hipSuccess && g) (void)hipGraphDestroy(g);
            return rc;
        }
        HIPCHK(e);
        book->graph = g;
        HIPCHK(hipGraphInstantiate(&book->gexec, g, nullptr, nullptr, 0));
        book->g_out = d_out;
        book->g_grad = d_grad;
        book->g_nt = nt;
    }
    HIPCHK(hipGraphLaunch(book->gexec, (hipStream_t)stream));
    return BT_OK;
}

}  // namespace

namespace {

// Batch workspaces, one per (device, stream, number type), kept until
// bt_shutdown.
struct WsEntry {
    int device;
    hipStream_t stream;
    bool greeks;
    bt_book *ws;
};
std::mutex g_ws_mu;
std::vector<WsEntry> g_ws;

bool same_tune(const bt_tune &x, const bt_tune &y)
{
    return x.wgs_per_cu == y.wgs_per_cu && x.level_factor == y.level_factor && x.pool_points == y.pool_points &&
           x.band_levels == y.band_levels && x.flags == y.flags;
}

// The workspace for a call of n options with N up to max_N on `stream`;
// (re)built when there is none or it is too small or differently tuned.
int batch_workspace(hipStream_t stream, int n, int max_N, const bt_tune *tune, bool greeks, bt_book **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const bt_tune t = batch_tune(tune, greeks);
    WsEntry *e = nullptr;
    for (WsEntry &w : g_ws)
        if (w.device == dev && w.stream == stream && w.greeks == greeks) e = &w;
    if (e && e->ws->cap_n >= n && e->ws->cap_N >= max_N && same_tune(e->ws->tune, t)) {
        *out = e->ws;
        return BT_OK;
    }
    // growing allocates and waits for the device: not allowed under capture
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return BT_ENOSUPP;
    int cap_n = n, cap_N = max_N;
    if (e) {
        if (same_tune(e->ws->tune, t)) {
            cap_n = std::max(cap_n, e->ws->cap_n);
            cap_N = std::max(cap_N, e->ws->cap_N);
        }
        bt_book_destroy(e->ws);
        e->ws = nullptr;
    }
    bt_book *b = new (std::nothrow) bt_book();
    if (!b) return BT_ENOMEM;
    Carver cv;
    const int rc = batch_build(b, cap_n, cap_N, t, 0, (int64_t)1 << 31, cv);
    if (rc != BT_OK) {
        book_free(b);
        delete b;
        if (e) g_ws.erase(g_ws.begin() + (e - g_ws.data()));
        return rc;
    }
    if (e) e->ws = b;
    else g_ws.push_back(WsEntry{dev, stream, greeks, b});
    *out = b;
    return BT_OK;
}

// The device array behind bt_price_batch_static: every buffer of its
// workspace is carved out of it, so that entry point allocates nothing.
// Each GPU holds its own copy until the process ends; in host code the name
// is only a stand-in, its device address comes from hipGetSymbolAddress.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
struct StaticWs {
    void *ptr = nullptr;       // this device's address of `scratch`
    bt_book *ws = nullptr;     // the workspace carved out of it
};
std::mutex g_static_mu;
StaticWs g_static[MAX_DEVICES];

// Set-up on the current device, once: the scratch array's device address,
// then the workspace carved from it (bt.h: BT_STATIC_MAX_OPTIONS options of
// up to BT_STATIC_MAX_N steps, 32 persistent workgroups per party, the
// recursions one after the other on the caller's stream).
int static_workspace(bt_book **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return BT_ENOSUPP;
    StaticWs &e = g_static[dev];
    if (e.ws) {
        *out = e.ws;
        return BT_OK;
    }
    if (!e.ptr) {
        void *p = nullptr;
        const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !p) {
            g_last_hip = (int)err;
            return BT_EHIP;
        }
        e.ptr = p;
    }
    bt_book *b = new (std::nothrow) bt_book();
    if (!b) return BT_ENOMEM;
    b->carved = true;
    Carver cv;
    cv.base = (char *)e.ptr;
    cv.cap = STATIC_SCRATCH_BYTES;
    bt_tune t = batch_tune(nullptr, false);
    t.level_factor = 8;
    t.pool_points = 16384;
    const int rc = batch_build(b, BT_STATIC_MAX_OPTIONS, BT_STATIC_MAX_N, t, 32, (int64_t)1 << 22, cv, 0, false);
    if (rc != BT_OK) {
        book_free(b);
        delete b;
        return rc;
    }
    e.ws = b;
    *out = b;
    return BT_OK;
}

// Workspace of the reverse-mode Greeks: the per-workgroup buffers of
// adjoint_tree, for tree sides of up to cap_N steps, on as many workgroups
// as fit a budget of device memory (at most one per compute unit).
struct AdjWs {
    int device = 0;
    hipStream_t stream = nullptr;
    int cap_n = 0, cap_N = 0, grid = 0, grid_p0 = 0;
    double *d_ws = nullptr;
    int *d_wsi = nullptr;
    // the device planner's constants and order, and the zero-cost kernel's
    // buffers, for cap_n options
    Model *d_models = nullptr;
    int2 *d_keys = nullptr;
    int *d_order = nullptr;
    int *d_ints = nullptr;          // valid count, queues, zero-cost queue
    unsigned long long *d_ctr = nullptr;
    double *d_wsp = nullptr;
    AdjArgs args{};
    KArgs k{};
    PlanArgs plan{};
};
std::vector<AdjWs *> g_adj;

void adj_free(AdjWs *w)
{
    if (!w) return;
    void *ptrs[] = {w->d_ws, w->d_wsi, w->d_models, w->d_keys, w->d_order, w->d_ints, w->d_ctr, w->d_wsp};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete w;
}

int adj_build(AdjWs *w, int cap_n, int cap_N)
{
    AdjArgs a{};
    const int64_t NN = cap_N + 2;
    const int B = 4 * cap_N + 64;
    const int s = isqrt_ceil(cap_N + 2);
    a.Ncap = cap_N;
    a.big_pts = B;
    // a level slot holds 32 points per node on average (a book's default
    // level factor) plus three large nodes
    a.lwn = round_up((3 * DEFAULT_LEVEL_FACTOR + 1) * NN + 6 * (int64_t)B, 32);
    a.cp_max = s + 2;
    a.sg_max = s;
    a.cp_nums = round_up((int64_t)a.cp_max * a.lwn / 2, 32);
    a.sg_nums = round_up((int64_t)a.sg_max * a.lwn / 2, 32);
    a.lane_doubles = stepper_doubles(2 * ADJ_LANE_PTS + 16, ADJ_LANE_PTS, ADJ_LANE_TAPE);
    a.big_doubles = stepper_doubles(2 * B + 16, B, 40 * B + 4096);
    a.oStab = 0;
    a.oSfac = round_up(2 * NN, 32);
    a.oW0 = a.oSfac + round_up(2 * NN, 32);
    a.oW1 = a.oW0 + a.lwn;
    a.oA0 = a.oW1 + a.lwn;
    a.oA1 = a.oA0 + a.lwn;
    a.oCP = a.oA1 + a.lwn;
    a.oSG = a.oCP + a.cp_nums;
    a.oLane = a.oSG + a.sg_nums;
    a.oBig = a.oLane + (int64_t)WG * a.lane_doubles;
    a.ws_doubles = a.oBig + NWAVE * a.big_doubles;
    a.iW0 = 0;
    a.iW1 = 2 * NN;
    a.iCP = 4 * NN;
    a.iSG = a.iCP + 2 * NN * a.cp_max;
    a.iTab = round_up(a.iSG + 2 * NN * a.sg_max, 2);
    a.wsi_ints = round_up(a.iTab + 2 * (int64_t)(a.cp_max + 1 + a.sg_max), 64);
    if (a.lwn > INT32_MAX || a.cp_nums > INT32_MAX || a.sg_nums > INT32_MAX || 40 * (int64_t)B + 4096 > INT32_MAX)
        return BT_EINVAL;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = (size_t)1 << 34;
    }
    const double per_wg = (double)a.ws_doubles * 8 + (double)a.wsi_ints * 4;
    const double budget = std::min((double)free_b / 3.0, 48.0 * (1 << 30));
    const int grid = (int)std::max(1.0, std::min((double)prop.multiProcessorCount, budget / per_wg));
    const int grid_p0 = std::max(1, std::min(cap_n, prop.multiProcessorCount));
    KArgs k{};
    k.p0_stab = round_up(2 * NN - 1, 32);
    k.p0_doubles = k.p0_stab + round_up(2 * NN - 2, 32);
    int rc = BT_OK;
    if ((rc = dalloc(&w->d_ws, (size_t)a.ws_doubles * grid)) || (rc = dalloc(&w->d_wsi, (size_t)a.wsi_ints * grid)) ||
        (rc = dalloc(&w->d_models, cap_n)) || (rc = dalloc(&w->d_keys, cap_n)) ||
        (rc = dalloc(&w->d_order, 3 * (size_t)cap_n)) || (rc = dalloc(&w->d_ints, 72)) ||
        (rc = dalloc(&w->d_ctr, 2)) || (rc = dalloc(&w->d_wsp, (size_t)k.p0_doubles * grid_p0)))
        return rc;
    a.ws = w->d_ws;
    a.wsi = w->d_wsi;
    a.models = w->d_models;
    a.count = w->d_ints;
    a.queue = w->d_ints + 2;          // zeroed by the reset kernel (its band counters)
    k.models = w->d_models;
    k.band_ctr = w->d_ints + 2;
    k.nbands_max = 1;
    k.arena_ctr = w->d_ctr;
    k.p0_queue = w->d_ints + 8;
    k.p0_count = w->d_ints;
    k.wsp = w->d_wsp;
    PlanArgs P{};
    P.models = w->d_models;
    P.keys = w->d_keys;
    P.order = w->d_order;
    P.count = w->d_ints;
    w->args = a;
    w->k = k;
    w->plan = P;
    w->cap_n = cap_n;
    w->cap_N = cap_N;
    w->grid = grid;
    w->grid_p0 = grid_p0;
    w->device = dev;
    return BT_OK;
}

int adjoint_workspace(hipStream_t stream, int n, int max_N, AdjWs **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    AdjWs *e = nullptr;
    size_t ei = 0;
    for (size_t i = 0; i < g_adj.size(); i++)
        if (g_adj[i]->device == dev && g_adj[i]->stream == stream) { e = g_adj[i]; ei = i; }
    if (e && e->cap_N >= max_N && e->cap_n >= n) {
        *out = e;
        return BT_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return BT_ENOSUPP;
    int cap_n = n, cap_N = max_N;
    if (e) {
        cap_n = std::max(cap_n, e->cap_n);
        cap_N = std::max(cap_N, e->cap_N);
        HIPCHK(hipDeviceSynchronize());
        adj_free(e);
        g_adj.erase(g_adj.begin() + ei);
    }
    AdjWs *w = new (std::nothrow) AdjWs();
    if (!w) return BT_ENOMEM;
    const int rc = adj_build(w, cap_n, cap_N);
    if (rc != BT_OK) {
        adj_free(w);
        return rc;
    }
    w->stream = stream;
    g_adj.push_back(w);
    *out = w;
    return BT_OK;
}

// Prices, counts and reverse-mode Greeks of a device-resident batch: the
// device planner's constants and order, the zero-cost kernel, then the
// buyer's and the seller's reverse sweeps, all on the caller's stream.
int price_adjoint(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, bt_grad *d_grad,
                  void *stream)
{
    if (n < 0 || max_N < 1 || max_N > BT_MAX_N || (n > 0 && (!d_params || !d_out || !d_grad))) return BT_EINVAL;
    if (n == 0) return BT_OK;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    hipStream_t s = (hipStream_t)stream;
    AdjWs *aw = nullptr;
    int rc = adjoint_workspace(s, n, max_N, &aw);
    if (rc != BT_OK) return rc;
    PlanArgs P = aw->plan;
    P.params = d_params;
    P.n = n;
    P.max_N = max_N;
    KArgs a = aw->k;
    a.out = d_out;
    a.grad = d_grad;
    a.n_opts = n;
    a.n_items = 0;
    a.p0_sched = aw->d_order + 2 * (int64_t)n;
    const int g1 = (n + WG - 1) / WG;
    hipLaunchKernelGGL(bt_derive_kernel, dim3(g1), dim3(WG), 0, s, P);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(bt_rank_kernel, dim3(g1), dim3(WG), 0, s, P);
    HIPCHK(hipGetLastError());
    const int rb = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(bt_reset_kernel, dim3(rb), dim3(256), 0, s, a, (int64_t)0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(bt_price0_kernel, dim3(std::min(aw->grid_p0, n)), dim3(WG), 0, s, a);
    HIPCHK(hipGetLastError());
    AdjArgs A = aw->args;
    A.out = d_out;
    A.grad = d_grad;
    const int gb = std::min(aw->grid, n);
    A.order = aw->d_order;   // the buyer's order: costly tree sides first
    hipLaunchKernelGGL(bt_adjoint_kernel<1>, dim3(gb), dim3(WG), 0, s, A);
    HIPCHK(hipGetLastError());
    A.order = aw->d_order + n;
    hipLaunchKernelGGL(bt_adjoint_kernel<0>, dim3(gb), dim3(WG), 0, s, A);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(bt_finalize_kernel, dim3((int)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
    return BT_OK;
}

int price_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, bt_grad *d_grad, void *stream,
                const bt_tune *tune)
{
    if (n < 0 || max_N < 1 || max_N > BT_MAX_N || (n > 0 && (!d_params || !d_out))) return BT_EINVAL;
    if (tune && tune->band_levels != 0 && (tune->band_levels < MIN_BAND || tune->band_levels > BAND)) return BT_EINVAL;
    if (n == 0) return BT_OK;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    bt_book *ws = nullptr;
    const int rc = batch_workspace((hipStream_t)stream, n, max_N, tune, d_grad != nullptr, &ws);
    if (rc != BT_OK) return rc;
    return d_grad ? launch_all<D4>(ws, d_out, d_grad, stream, d_params, n, max_N)
                  : launch_all<double>(ws, d_out, nullptr, stream, d_params, n, max_N);
}

}  // namespace

extern "C" {

int bt_book_price(bt_book *book, bt_result *d_out, void *stream)
{
    if (!book || !d_out) return BT_EINVAL;
    return launch<double>(book, d_out, nullptr, stream);
}

int bt_book_price_hedge(bt_book *book, bt_result *d_out, bt_hedge *d_hedge, void *stream)
{
    if (!book || !d_out || !d_hedge || book->device_plan) return BT_EINVAL;
    return launch_all<double>(book, d_out, nullptr, stream, nullptr, 0, 0, d_hedge);
}

int bt_book_price_exercise(bt_book *book, bt_result *d_out, uint8_t *d_map, void *stream)
{
    if (!book || !d_out || !d_map || book->device_plan) return BT_EINVAL;
    if (!book->d_exoff) {
        // option i's seller plane from off[i], its buyer plane after it
        std::vector<int64_t> off(book->n + 1, 0);
        for (int i = 0; i < book->n; i++) {
            const int64_t N = book->params[i].N;
            off[i + 1] = off[i] + (N >= 1 && N <= BT_MAX_N ? (N + 1) * (N + 2) : 0);
        }
        int64_t *d = nullptr;
        HIPCHK(hipMalloc(&d, sizeof(int64_t) * off.size()));
        const hipError_t e = hipMemcpy(d, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            HIPCHK(e);
        }
        book->d_exoff = d;
    }
    return launch_all<double>(book, d_out, nullptr, stream, nullptr, 0, 0, nullptr, d_map);
}

int bt_book_price_grad(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream)
{
    if (!book || !d_out || !d_grad) return BT_EINVAL;
    if (!book->greeks) return BT_ENOSUPP;
    return launch<D4>(book, d_out, d_grad, stream);
}

int bt_price_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, void *stream,
                   const bt_tune *tune)
{
    return price_batch(d_params, n, max_N, d_out, nullptr, stream, tune);
}

int bt_price_batch_static(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, void *stream)
{
    if (n < 0 || n > BT_STATIC_MAX_OPTIONS || max_N < 1 || max_N > BT_STATIC_MAX_N || (n > 0 && (!d_params || !d_out)))
        return BT_EINVAL;
    if (n == 0) return BT_OK;
    std::lock_guard<std::mutex> lock(g_static_mu);
    bt_book *ws = nullptr;
    const int rc = static_workspace(&ws);
    if (rc != BT_OK) return rc;
    return launch_all<double>(ws, d_out, nullptr, stream, d_params, n, max_N);
}

int bt_price_adjoint_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, bt_grad *d_grad,
                           void *stream)
{
    return price_adjoint(d_params, n, max_N, d_out, d_grad, stream);
}

int bt_price_grad_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, bt_grad *d_grad,
                        void *stream, const bt_tune *tune)
{
    if (n > 0 && !d_grad) return BT_EINVAL;
    return price_batch(d_params, n, max_N, d_out, d_grad, stream, tune);
}

int bt_book_resolve_overflow(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream,
                             int32_t *remaining)
{
    if (!book || !d_out) return BT_EINVAL;
    if (d_grad && !book->greeks) return BT_ENOSUPP;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    std::vector<bt_result> res(book->n);
    HIPCHK(hipMemcpy(res.data(), d_out, sizeof(bt_result) * book->n, hipMemcpyDeviceToHost));
    std::vector<int> idx;
    for (int i = 0; i < book->n; i++)
        if (res[i].status == BT_EOVERFLOW) idx.push_back(i);
    std::vector<bt_grad> grd;
    if (d_grad && !idx.empty()) {
        grd.resize(book->n);
        HIPCHK(hipMemcpy(grd.data(), d_grad, sizeof(bt_grad) * book->n, hipMemcpyDeviceToHost));
    }
    const int base_lf = book->tune.level_factor > 0 ? book->tune.level_factor : DEFAULT_LEVEL_FACTOR;
    const int64_t base_pool = book->tune.pool_points > 0 ? book->tune.pool_points
                                                         : (book->greeks ? DEFAULT_POOL_POINTS / 4 : DEFAULT_POOL_POINTS);
    const bool had = !idx.empty();
    // prices the options ids with level buffers `mult` times the book's;
    // a set whose book does not fit in device memory is halved (a single
    // option that does not fit stays overflowed)
    std::vector<int> still;
    const std::function<int(const std::vector<int> &, int)> price_set = [&](const std::vector<int> &ids,
                                                                            int mult) -> int {
        std::vector<bt_params> sub;
        int sub_N = 1;
        for (int i : ids) {
            sub.push_back(book->params[i]);
            sub_N = std::max(sub_N, (int)book->params[i].N);
        }
        bt_tune t = book->tune;
        t.flags = d_grad ? BT_TUNE_GREEKS : 0;
        t.level_factor = base_lf * mult;
        // a level that large would need offsets beyond int: these stay overflowed
        if ((int64_t)t.level_factor * (sub_N + 2) * 3 + (sub_N + 2) > INT32_MAX) {
            still.insert(still.end(), ids.begin(), ids.end());
            return BT_OK;
        }
        t.pool_points = (int32_t)std::min<int64_t>(base_pool * mult, (int64_t)1 << 22);
        t.wgs_per_cu = 1;
        bt_book *sb = nullptr;
        int rc = bt_book_create(sub.data(), (int32_t)sub.size(), &t, &sb);
        bt_result *d_sub = nullptr;
        bt_grad *d_subg = nullptr;
        if (rc == BT_OK && (hipMalloc(&d_sub, sizeof(bt_result) * sub.size()) != hipSuccess ||
                            (d_grad && hipMalloc(&d_subg, sizeof(bt_grad) * sub.size()) != hipSuccess))) {
            (void)hipGetLastError();
            rc = BT_ENOMEM;
        }
        const bool no_room = rc == BT_ENOMEM || (rc == BT_EHIP && g_last_hip == (int)hipErrorOutOfMemory);
        if (rc != BT_OK) {
            if (d_sub) (void)hipFree(d_sub);
            if (sb) bt_book_destroy(sb);
            if (!no_room) return rc;
            (void)hipGetLastError();
            if (ids.size() == 1) {
                still.push_back(ids[0]);
                return BT_OK;
            }
            const size_t h = ids.size() / 2;
            const int r1 = price_set(std::vector<int>(ids.begin(), ids.begin() + h), mult);
            if (r1 != BT_OK) return r1;
            return price_set(std::vector<int>(ids.begin() + h, ids.end()), mult);
        }
        rc = d_grad ? bt_book_price_grad(sb, d_sub, d_subg, stream) : bt_book_price(sb, d_sub, stream);
        std::vector<bt_result> sres(sub.size());
        std::vector<bt_grad> sgrd(d_grad ? sub.size() : 0);
        if (rc == BT_OK) {
            hipError_t e = hipMemcpyAsync(sres.data(), d_sub, sizeof(bt_result) * sub.size(), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && d_grad)
                e = hipMemcpyAsync(sgrd.data(), d_subg, sizeof(bt_grad) * sub.size(), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { g_last_hip = (int)e; rc = BT_EHIP; }
        }
        (void)hipFree(d_sub);
        if (d_subg) (void)hipFree(d_subg);
        bt_book_destroy(sb);
        if (rc != BT_OK) return rc;
        for (size_t j = 0; j < ids.size(); j++) {
            res[ids[j]] = sres[j];
            if (d_grad) grd[ids[j]] = sgrd[j];
            if (sres[j].status == BT_EOVERFLOW) still.push_back(ids[j]);
        }
        return BT_OK;
    };
    for (int mult = 4; !idx.empty() && mult <= 1024; mult *= 4) {
        still.clear();
        const int rc = price_set(idx, mult);
        if (rc != BT_OK) return rc;
        std::sort(still.begin(), still.end());
        idx.swap(still);
    }
    if (had) {
        HIPCHK(hipMemcpyAsync(d_out, res.data(), sizeof(bt_result) * book->n, hipMemcpyHostToDevice, s));
        if (d_grad)
            HIPCHK(hipMemcpyAsync(d_grad, grd.data(), sizeof(bt_grad) * book->n, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (remaining) *remaining = (int32_t)idx.size();
    return BT_OK;
}

int bt_book_timings(bt_book *book, double *ms, int32_t *calls)
{
    if (!book || !ms) return BT_EINVAL;
    if (!book->timing) return BT_ENOSUPP;
    for (int i = 0; i < BT_NUM_KERNELS; i++) ms[i] = 0.0;
    const size_t nc = book->events.size() / NEV;
    // (start, end) events of setup, buyer, seller, zero-cost
    const int pair[BT_NUM_KERNELS][2] = {{0, 1}, {1, 2}, {3, 4}, {5, 6}};
    int rc = BT_OK;
    for (size_t c = 0; c < nc; c++) {
        hipEvent_t *e = &book->events[c * NEV];
        for (int i = 0; i < NEV; i++)
            if (hipEventSynchronize(e[i]) != hipSuccess) rc = BT_EHIP;
        for (int i = 0; i < BT_NUM_KERNELS && rc == BT_OK; i++) {
            float t = 0.0f;
            hipError_t err = hipEventElapsedTime(&t, e[pair[i][0]], e[pair[i][1]]);
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

int bt_autotune(const bt_params *h_params, int32_t n, const bt_tune *base, const bt_tune *cand, int32_t n_cand,
                int32_t reps, void *stream, bt_tune *best, double *ms)
{
    if (!h_params || n < 1 || !best || reps < 1 || (cand && n_cand < 1)) return BT_EINVAL;
    std::vector<bt_tune> list;
    const bt_tune b0 = base ? *base : bt_tune{};
    if (cand) {
        list.assign(cand, cand + n_cand);
    } else {
        for (int band : {8, 16, 32})
            for (int w : {1, 2}) {
                bt_tune t = b0;
                t.band_levels = band;
                t.wgs_per_cu = w;
                list.push_back(t);
            }
    }
    hipStream_t s = (hipStream_t)stream;
    bt_result *d_out = nullptr;
    bt_grad *d_grad = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BT_OK, best_i = -1;
    double best_ms = 0.0;
    auto hip_ok = [&](hipError_t e) {
        if (e == hipSuccess) return true;
        g_last_hip = (int)e;
        rc = BT_EHIP;
        return false;
    };
    if (hip_ok(hipMalloc(&d_out, (size_t)n * sizeof(bt_result))) &&
        hip_ok(hipMalloc(&d_grad, (size_t)n * sizeof(bt_grad))) && hip_ok(hipEventCreate(&e0)) &&
        hip_ok(hipEventCreate(&e1))) {
        for (size_t i = 0; i < list.size() && rc == BT_OK; i++) {
            bt_tune t = list[i];
            t.flags &= ~(BT_TUNE_TIMING | BT_TUNE_GRAPH);
            const bool grad = (t.flags & BT_TUNE_GREEKS) != 0;
            if (ms) ms[i] = -1.0;
            bt_book *bk = nullptr;
            const int crc = bt_book_create(h_params, n, &t, &bk);
            if (crc == BT_EINVAL) continue;   // a candidate the library rejects
            if (crc != BT_OK) { rc = crc; break; }
            auto call = [&]() { return grad ? bt_book_price_grad(bk, d_out, d_grad, s) : bt_book_price(bk, d_out, s); };
            int prc = call();
            if (prc == BT_OK && hip_ok(hipEventRecord(e0, s))) {
                for (int r = 0; r < reps && prc == BT_OK; r++) prc = call();
                if (prc == BT_OK && hip_ok(hipEventRecord(e1, s)) && hip_ok(hipEventSynchronize(e1))) {
                    float el = 0.0f;
                    if (hip_ok(hipEventElapsedTime(&el, e0, e1))) {
                        const double m = el / reps;
                        if (ms) ms[i] = m;
                        if (best_i < 0 || m < best_ms) { best_ms = m; best_i = (int)i; }
                    }
                }
            }
            if (prc != BT_OK && rc == BT_OK) rc = prc;
            bt_book_destroy(bk);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_out) (void)hipFree(d_out);
    if (d_grad) (void)hipFree(d_grad);
    if (rc != BT_OK) return rc;
    if (best_i < 0) return BT_EINVAL;
    *best = list[best_i];
    return BT_OK;
}

int bt_price(const bt_params *p, bt_result *out)
{
    if (!p || !out) return BT_EINVAL;
    // one cached book per thread, rebuilt when N changes (the band tasks
    // depend on N only); otherwise only the option's constants are replaced
    bt_result *&d_res = t_price_res;
    bt_book *&cache = t_price_book;
    int &cache_N = t_price_N;
    if (!d_res) HIPCHK(hipMalloc(&d_res, sizeof(bt_result)));
    Model m;
    const bool ok = derive(*p, m);
    int rc = BT_OK;
    if (cache && ok && cache_N == p->N && cache->n_items > 0) {
        HIPCHK(hipMemcpy(cache->d_models, &m, sizeof(Model), hipMemcpyHostToDevice));
        cache->params[0] = *p;
    } else {
        if (cache) { bt_book_destroy(cache); cache = nullptr; cache_N = -1; }
        rc = bt_book_create(p, 1, nullptr, &cache);
        if (rc != BT_OK) return rc;
        cache_N = ok ? p->N : -1;
    }
    rc = bt_book_price(cache, d_res, nullptr);
    if (rc == BT_OK) rc = bt_book_resolve_overflow(cache, d_res, nullptr, nullptr, nullptr);
    if (rc != BT_OK) return rc;
    HIPCHK(hipMemcpy(out, d_res, sizeof(bt_result), hipMemcpyDeviceToHost));
    return BT_OK;
}

int bt_shutdown(void)
{
    {
        std::lock_guard<std::mutex> lock(g_ws_mu);
        int cur = 0;
        const bool have_dev = hipGetDevice(&cur) == hipSuccess;
        for (WsEntry &w : g_ws) {
            if (hipSetDevice(w.device) == hipSuccess) bt_book_destroy(w.ws);
        }
        g_ws.clear();
        for (AdjWs *w : g_adj) {
            if (hipSetDevice(w->device) == hipSuccess) {
                (void)hipDeviceSynchronize();
                adj_free(w);
            }
        }
        g_adj.clear();
        if (have_dev) (void)hipSetDevice(cur);
    }
    if (t_price_book) {
        bt_book_destroy(t_price_book);
        t_price_book = nullptr;
    }
    t_price_N = -1;
    if (t_price_res) {
        (void)hipFree(t_price_res);
        t_price_res = nullptr;
    }
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
