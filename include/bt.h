/*
 * bt.h -- C ABI of libbtprice: ask and bid prices of American options under
 * proportional transaction costs on a recombining CRR binomial tree, and the
 * zero-cost CRR price, computed on one AMD Instinct MI355X (gfx950).
 *
 * Method: Zhang, Roux & Zastawniak, "Parallel Binomial American Option
 * Pricing with (and without) Transaction Costs" (2011).
 *   - Tree model (Section 4.1): N steps, u = exp(sigma sqrt(T/N)), d = 1/u,
 *     r = exp(R T/N); bid/ask stock prices (1 -+ k) S (Section 3); an extra
 *     time N+1 with payoff (0, 0); no transaction cost at t = 0.
 *   - Seller (ask) and buyer (bid) backward induction over piecewise-linear
 *     expense functions of the stock holding (Section 3): w = max of the two
 *     successors, v = w / r with slopes restricted to [-S^a_t, -S^b_t],
 *     z = max(u_t, v) for the seller, min(u_t, v) for the buyer;
 *     ask = z_0(0), bid = -z_0(0).
 *   - Zero-cost price (Section 3 and Appendix): scalar CRR recursion without
 *     the extra time step.
 *
 * Conventions shared by every entry point:
 *   - Plain C types only; nothing crosses the ABI that a C caller cannot
 *     build.  No exceptions escape.
 *   - Return value: BT_OK (0) or a negative BT_E* code.  bt_strerror() names
 *     it; after BT_EHIP, bt_last_hip_error() returns the hipError_t value of
 *     the failing HIP call on the calling thread.
 *   - "host pointer" arguments are read or written synchronously before the
 *     call returns; "device pointer" arguments must point to device memory of
 *     the current HIP device and are accessed asynchronously on `stream`
 *     (a hipStream_t passed as void*, NULL = the null stream).
 *   - All memory passed in is owned by the caller.  The library owns only
 *     what a book (bt_book) allocates, freed by bt_book_destroy(), and the
 *     workspaces of bt_price, bt_price_batch and bt_price_grad_batch, freed
 *     by bt_shutdown().
 *   - All arithmetic is IEEE binary64 with no contraction.
 */
#ifndef BT_H
#define BT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BT_VERSION 10000 /* 1.0.0 */

/* Error codes. */
#define BT_OK 0
#define BT_EINVAL (-1)    /* invalid argument or option parameters          */
#define BT_ENOMEM (-2)    /* device or host allocation failed               */
#define BT_EHIP (-3)      /* a HIP runtime call failed                      */
#define BT_EOVERFLOW (-4) /* a tree level exceeded the book's work buffers  */
#define BT_ENOSUPP (-5)   /* feature not supported                          */

/* Payoff processes (xi_t, zeta_t) of Section 3: the holder who exercises at
 * t receives xi_t in cash and zeta_t shares (settlement by delivery of the
 * stock or in cash).
 *   BT_PUT      : (K, -1), physical delivery (Section 3's example)
 *   BT_CALL     : (-K, 1), physical delivery
 *   BT_BULL     : ((S-K)^+ - (S-K2)^+, 0), cash settled (Section 5's bull
 *                 spread; K2 > K)
 *   BT_PUT_CASH : ((K-S)^+, 0), cash settled
 *   BT_CALL_CASH: ((S-K)^+, 0), cash settled
 *   BT_BEAR     : ((K2-S)^+ - (K-S)^+, 0), cash settled (K2 > K)
 *   BT_STRADDLE : (|S-K|, 0), cash settled
 * With costs the settlement matters: a delivered put or call trades the
 * share at exercise, a cash-settled one does not.  At k = 0 both give the
 * same prices. */
enum { BT_PUT = 0, BT_CALL = 1, BT_BULL = 2, BT_PUT_CASH = 3, BT_CALL_CASH = 4, BT_BEAR = 5, BT_STRADDLE = 6 };

/* Option flags.
 *   BT_F_EUROPEAN   exercise only at N (test variant; z_t = v_t for t < N)
 *   BT_F_COST_AT_T0 charge the cost rate k at t = 0 as well (the paper's
 *                   model charges none at t = 0, Section 4.1)              */
enum { BT_F_EUROPEAN = 1u, BT_F_COST_AT_T0 = 2u };

/* One option.  S0, K, sigma, T > 0; K2 > K for BT_BULL and BT_BEAR
 * (ignored otherwise);
 * R is the continuously compounded annual rate; 0 <= k < 1;
 * 1 <= N <= BT_MAX_N; the tree must be free of arbitrage: d < r < u. */
typedef struct {
    double S0, K, K2, R, sigma, T, k;
    int32_t N, payoff;
    uint32_t flags, reserved; /* reserved must be 0 */
} bt_params;

#define BT_MAX_N 65536

/* Result of one option.  ask/bid: the Section 3 prices; price0: the
 * zero-cost CRR price.  bp_*: breakpoint statistics of the expense functions
 * z_t over all nodes of levels 0..N of one side (a breakpoint is a change of
 * slope); status: BT_OK or the error of this option (prices are NaN then). */
typedef struct {
    double ask, bid, price0;
    int64_t bp_total_ask, bp_total_bid;
    int32_t bp_max_ask, bp_max_bid;
    int32_t status, reserved;
} bt_result;

/* Derivatives of ask and bid with respect to S0, sigma, R and k, taken on
 * the active branch of the piecewise-smooth price (N, T, K, K2 fixed). */
typedef struct {
    double dS0, dsigma, dR, dk;
} bt_grad4;
typedef struct {
    bt_grad4 ask, bid;
} bt_grad;

/* The optimal stock holdings at t = 0 -- the hedges of the two parties
 * (Section 3: the root's slope restriction is the cheapest rebalancing from
 * no shares, v_0(0) = min over y of f(y) + S^a_0 y^+ - S^b_0 y^-, with
 * f = rho max(z_1(1), z_1(0)) of the party).  [ask_lo, ask_hi]: the
 * holdings the seller carries from t = 0 to t = 1 in an optimal superhedge
 * of the ask; [bid_lo, bid_hi]: the buyer's.  The minimum is attained at a
 * breakpoint of f or at 0; the interval spans the candidates within 1e-12
 * (relative, floor 1) of it, a single point unless a piece is flat.  At
 * k = 0 the seller holds the CRR delta and the buyer its opposite. */
typedef struct {
    double ask_lo, ask_hi, bid_lo, bid_hi;
} bt_hedge;

/* Launch tuning; pass NULL for the library's choice.  Zero fields also mean
 * "library's choice".
 *   wgs_per_cu   persistent workgroups per compute unit (default 2)
 *   level_factor capacity of one tree level, in points per node (default
 *                32); a workgroup's private level holds at least
 *                65536 * max(1, level_factor / 32) points, and 16N for a
 *                book with the buyer of a call or a bull spread with costs
 *                at N steps
 *   pool_points  per-workgroup temporaries of the nodes with many
 *                breakpoints, in points (default 262144; 65536 for a
 *                BT_TUNE_GREEKS book); a node too big for its wave's share
 *                takes its temporaries from its party's arena instead.
 *                bt_book_create sizes each party's arena from the book's
 *                options (the buyer sides of calls and bull spreads with
 *                costs, which grow the largest nodes): at least 2^28
 *                doubles (5x that for Greeks, and at least 64 pools), at
 *                most 2^32 doubles or an eighth of the free device memory.
 *                Options whose nodes outgrow it end BT_EOVERFLOW, for
 *                bt_book_resolve_overflow
 *   flags        BT_TUNE_TIMING: record HIP events around every kernel of
 *                every pricing call (read with bt_book_timings; not for use
 *                under graph capture);
 *                BT_TUNE_GREEKS: size the book's buffers for
 *                bt_book_price_grad (values with four tangents, 5x the
 *                memory of a price-only book);
 *                BT_TUNE_GRAPH: the first pricing call with given output
 *                buffers captures the book's whole launch sequence into a
 *                HIP graph (on a stream of the book's own); that call and
 *                the later ones with the same buffers launch the graph on
 *                the caller's stream.  New buffers re-capture.  No HIP
 *                events are recorded in this mode (BT_TUNE_TIMING is
 *                ignored)
 *   band_levels  tree levels per band launch, 2..32 (default 32): a band's
 *                column blocks are 256 - band_levels columns wide and each
 *                recomputes a halo of band_levels - 1 columns, so shorter
 *                bands recompute less and launch more often.  Outside
 *                2..32 (and not 0) bt_book_create returns BT_EINVAL.
 * No field changes a result: prices, Greeks and breakpoint counts are the
 * same bits under every tuning.                                            */
typedef struct {
    int32_t wgs_per_cu, level_factor, pool_points, flags, band_levels;
} bt_tune;

enum { BT_TUNE_TIMING = 1, BT_TUNE_GREEKS = 2, BT_TUNE_GRAPH = 4 };

/* Number of kernels one pricing call launches, in launch order:
 * 0 = result/queue reset, 1 = buyer (bid), 2 = seller (ask), 3 = zero-cost. */
#define BT_NUM_KERNELS 4

/* A book: a batch of options prepared for repeated pricing.  Creating it
 * validates every option (an invalid one gets status BT_EINVAL in every
 * result and is skipped by the kernels), derives the tree constants on the
 * host, orders the work longest-tree-first, and allocates every device
 * buffer the pricing calls need, so that bt_book_price and
 * bt_book_price_grad allocate nothing and can be captured in a HIP graph.
 * The book belongs to the HIP device that is current when it is created. */
typedef struct bt_book bt_book;

/* h_params: host pointer to n options (n >= 1).  tune: host pointer or
 * NULL.  *out receives the book.  Returns BT_OK even when some options are
 * invalid (see the per-option status); BT_EINVAL only for bad arguments,
 * including a tuning whose level buffers would need offsets beyond int
 * (level_factor x 3 (N_max+2) above 2^31 - 1). */
int bt_book_create(const bt_params *h_params, int32_t n, const bt_tune *tune, bt_book **out);

/* Number of options, largest N, and the number of tree nodes
 * sum_i (N_i+1)(N_i+2)/2 of the valid options. */
int bt_book_info(const bt_book *book, int32_t *n, int32_t *n_max, int64_t *nodes);

/* Prices every option of the book: ask, bid (Section 3 recursions) and
 * price0 (zero-cost recursion).  d_out: device pointer to n bt_result, in
 * book order.  Asynchronous on `stream` (the three recursions run on two
 * streams of the book's own as well, forked from `stream` and joined back
 * to it before the call's work ends there); the book's buffers are shared
 * by all calls on it, so calls on one book must not overlap.
 * An option whose tree outgrows the book's buffers on either side gets
 * status BT_EOVERFLOW, NaN prices and zero counts (no partial result).
 * Whether an option outgrows the big-node arena can depend on the order in
 * which the GPU schedules the workgroups of a launch (the arena is shared by
 * all tree sides of a party), so two calls may differ in which options end
 * BT_EOVERFLOW; every option that ends BT_OK has the same bits in every
 * call, and bt_book_resolve_overflow completes the others with those same
 * bits. */
int bt_book_price(bt_book *book, bt_result *d_out, void *stream);

/* As bt_book_price, and also the Greeks of ask and bid: d_grad is a device
 * pointer to n bt_grad (NaN for invalid options).  The derivatives are
 * carried forward through the same recursion as the prices (every number of
 * every expense function holds its value and its derivatives with respect
 * to S0, sigma, R and k), so they are exact for the active branch of the
 * piecewise-smooth price.  The book must have been created with
 * BT_TUNE_GREEKS (else BT_ENOSUPP). */
int bt_book_price_grad(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream);

/* Batch pricing of options held in device memory (for example a caller's
 * tensors): ask, bid and price0 of d_params[0..n-1] into d_out[0..n-1],
 * asynchronous on `stream`, with the same results as a book of the same
 * options and tuning (Section 3 recursions, Section 4.1 tree).
 *   d_params  device pointer to n bt_params (read on the stream);
 *   n         number of options (0: nothing is done);
 *   max_N     the largest N the call may meet, 1..BT_MAX_N; an option with
 *             N > max_N gets status BT_EINVAL.  It sizes the workspace and
 *             fixes the launch sequence (ceil((max_N+1)/band_levels) band
 *             launches per party), so a tight bound is faster;
 *   d_out     device pointer to n bt_result;
 *   tune      host pointer or NULL; wgs_per_cu defaults to 1 here, and
 *             BT_TUNE_TIMING and BT_TUNE_GRAPH are ignored (capture the
 *             caller's stream instead).
 * Everything runs on the GPU: the tree constants (bt_model.hpp's correctly
 * rounded exp, bit-equal to bt_model_constants), the order of the tree
 * sides and the band task lists are built by kernels, then the book's
 * kernels price them.  Nothing of the options is read by the host.
 * Workspace: the library keeps one per (device, stream, with or without
 * Greeks), sized for n options of up to max_N steps each (as if every option
 * were the costly buyer of a call: about 2 x 2 x (3 level_factor + 1)(max_N+2)
 * numbers of band buffers per option, plus per-workgroup levels, pools and
 * each party's arena of at most 2^31 doubles).  A call that fits the
 * existing workspace allocates nothing, waits for nothing on the host and
 * can be captured in a HIP graph; a call that needs a larger one (more
 * options, a larger max_N, another tuning) frees the old one after waiting
 * for the device and allocates, which is refused with BT_ENOSUPP while the
 * stream is capturing.  bt_shutdown frees every workspace.  Calls on one
 * stream share its workspace in stream order; calls from several host
 * threads are serialised by the library.
 * Errors: BT_EINVAL (bad arguments), BT_ENOMEM, BT_EHIP, BT_ENOSUPP; per
 * option, status BT_EINVAL (invalid option) or BT_EOVERFLOW (its tree
 * outgrew the workspace: price it again with a larger level_factor or
 * pool_points, or through a book and bt_book_resolve_overflow).  An option
 * whose status is not BT_OK has NaN prices and zero counts (no partial
 * results). */
int bt_price_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, void *stream,
                   const bt_tune *tune);

/* As bt_price_batch, and the Greeks of ask and bid into d_grad[0..n-1]
 * (device pointer; NaN where status is not BT_OK), carried forward through
 * the recursion as in bt_book_price_grad.  Its workspace is separate from
 * the price-only one and holds five numbers per number. */
int bt_price_grad_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, bt_grad *d_grad,
                        void *stream, const bt_tune *tune);

/* Prices and reverse-mode Greeks of a batch of options held in device
 * memory: ask, bid, price0 and breakpoint counts into d_out[0..n-1] (the
 * same bits as bt_price_batch) and d(ask, bid)/d(S0, sigma, R, k) into
 * d_grad[0..n-1], asynchronous on `stream`.  The Greeks come from a reverse
 * sweep through each tree (Section 3's recursion run backwards), not from
 * carried tangents: one workgroup sweeps one tree side forward from level
 * N+1, keeping every s-th level (s = ceil(sqrt(N+2))) as a checkpoint, then
 * goes back from the root segment by segment, recomputing the levels
 * between two checkpoints from the upper one and stepping the adjoint of
 * each level back to the level below it through every node's merge,
 * discount, slope restriction and exercise (each node recomputed on numbers
 * that record their operations, its record read backwards).  Memory per
 * tree side is O(sqrt(N)) levels instead of the N levels of the tree.
 * Derivatives are those of the branch of the piecewise-smooth price active
 * at the given parameters, as for bt_price_grad_batch (equal to its values
 * up to rounding).
 *   max_N  1..BT_MAX_N, bounds every option's N (larger: BT_EINVAL status);
 * Workspace: one per (device, stream), kept until bt_shutdown, sized for n
 * options and max_N: per workgroup two level slots and two adjoint slots of
 * 32 points per node on average plus three large nodes, checkpoint and
 * segment regions of half a slot per level they hold, the per-lane scratch
 * and four large-node slots (nodes whose children hold up to 4 max_N + 64
 * points), on at most one workgroup per compute unit and within a third of
 * the free device memory.  A call that fits the existing
 * workspace allocates nothing and can be captured; one that needs a larger
 * workspace is refused with BT_ENOSUPP while the stream is capturing.
 * Errors as bt_price_batch; an option whose levels or nodes outgrow the
 * workspace ends BT_EOVERFLOW with NaN prices and Greeks. */
int bt_price_adjoint_batch(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, bt_grad *d_grad,
                           void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: as
 * bt_price_batch (prices only, the library's tuning with level_factor 8 and
 * pool_points 16384), but every buffer comes from one device array of
 * BT_STATIC_SCRATCH_BYTES that the library defines; no call allocates or
 * frees device memory.  Each GPU the library runs on holds its own copy of
 * the array until the process ends.  Limits: n <= BT_STATIC_MAX_OPTIONS and
 * max_N <= BT_STATIC_MAX_N, else BT_EINVAL; 32 persistent workgroups per
 * party, and the seller, buyer and zero-cost recursions run one after the
 * other on `stream`.  Every call on a GPU shares that GPU's array (its
 * counters are cleared at the start of each call): calls that overlap on
 * one GPU -- on different streams, or from different threads without
 * ordering -- race and give wrong results.  Options that outgrow the array's
 * buffers end BT_EOVERFLOW with NaN prices. */
#define BT_STATIC_SCRATCH_BYTES (256u << 20)
#define BT_STATIC_MAX_OPTIONS 64
#define BT_STATIC_MAX_N 1024
int bt_price_batch_static(const bt_params *d_params, int32_t n, int32_t max_N, bt_result *d_out, void *stream);

/* As bt_book_price, and the hedges at t = 0 of every option into d_hedge
 * (device pointer to n bt_hedge, NaN where status is not BT_OK): the root
 * of each tree side recomputes its discounted maximum in its workgroup's
 * temporaries and minimises the rebalancing cost over its breakpoints.  Not
 * replayed from a graph (BT_TUNE_GRAPH does not apply). */
int bt_book_price_hedge(bt_book *book, bt_result *d_out, bt_hedge *d_hedge, void *stream);

/* As bt_book_price, and the exercise maps of both parties into d_map
 * (device memory, caller-owned): for every node (t, c), t = 0..N, one byte,
 * 1 where exercise attains the party's expense at zero stock holding and 0
 * elsewhere (Section 3: the seller's z_t is max(u_t, v_t), so 1 when
 * u_t(0) >= v_t(0); the buyer's is min(u_t, v_t), so 1 when u_t(0) <=
 * v_t(0); no exercise before N in the European variant).  At k = 0 both
 * maps are the zero-cost stopping region {xi + zeta S >= continuation}.
 * Layout, in book order: option i takes 2 P_i bytes, P_i = (N_i + 1)(N_i +
 * 2) / 2 (0 when N_i is outside 1..BT_MAX_N), the seller's plane then the buyer's,
 * node (t, c) at t (t + 1) / 2 + c of a plane; option i starts at the sum
 * of 2 P_j over j < i.  The planes of an option whose status is not BT_OK
 * are set to 0xff.  The first call allocates n + 1 offsets (8 bytes each)
 * kept with the book.  Not replayed from a graph; bt_book_resolve_overflow
 * does not write maps (price such options in a book of their own with a
 * larger level_factor). */
int bt_book_price_exercise(bt_book *book, bt_result *d_out, uint8_t *d_map, void *stream);

/* Completes a pricing call whose options overflowed the book's buffers
 * (status BT_EOVERFLOW: a tree whose band levels, private levels or
 * big-node temporaries outgrew what the book sized for them): waits for
 * `stream`, then re-prices those options on `stream` with level_factor and
 * pool_points 4x larger each attempt (up to 1024x),
 * writing their results into d_out.  d_grad is NULL after bt_book_price;
 * after bt_book_price_grad it is that call's Greeks buffer, and the
 * re-pricing then also writes the Greeks of those options.  *remaining (may
 * be NULL) receives the number of options still overflowing.  Synchronous;
 * allocates temporary device memory only when some option overflowed, one
 * re-pricing book at a time: a set of options whose book does not fit in
 * device memory is re-priced in halves, and a single option that does not
 * fit even alone stays BT_EOVERFLOW (counted in *remaining), as does an
 * option whose level buffers would need more than 2^31 - 1 numbers (offsets
 * are int: level_factor x 3 (N+2) must stay below that). */
int bt_book_resolve_overflow(bt_book *book, bt_result *d_out, bt_grad *d_grad, void *stream,
                             int32_t *remaining);

/* For a book created with BT_TUNE_TIMING: waits for every pricing call
 * made since the previous bt_book_timings call, writes into ms[0..3] the
 * total milliseconds of each group of kernels over those calls -- setup
 * (reset and level N+1), the buyer's bands, the seller's bands, the
 * zero-cost recursion; the last three run concurrently, each on a stream of
 * its own, forked from and joined back to the call's stream -- and into
 * *calls their number.  BT_ENOSUPP without the flag. */
int bt_book_timings(bt_book *book, double *ms, int32_t *calls);

/* Frees the book's device memory (synchronises the device first). */
void bt_book_destroy(bt_book *book);

/* Autotuner: picks the tuning of a batch by timing it on the GPU.  For every
 * candidate tuning it builds a book of the n options in h_params (host
 * memory), prices it once to warm up and then `reps` times on `stream`,
 * timed with HIP events around the timed calls, and destroys the book; the
 * fastest candidate is written to *best and, when ms is not NULL, each
 * candidate's mean milliseconds per call to ms[i].  Candidates: the n_cand
 * tunings in cand (host memory), or, when cand is NULL, the library's list
 * of BT_AUTOTUNE_CANDIDATES tunings: band_levels in {8, 16, 32} x
 * wgs_per_cu in {1, 2}, every other field taken from *base (NULL: all zero).
 * A candidate with BT_TUNE_GREEKS is timed with bt_book_price_grad,
 * otherwise with bt_book_price; BT_TUNE_TIMING and BT_TUNE_GRAPH are cleared
 * for the timing and kept in *best.  A candidate that bt_book_create rejects
 * gets ms[i] = -1 and is skipped.  Options that outgrow their level buffers
 * are timed as they are (re-pricing them is bt_book_resolve_overflow's job,
 * outside the tuner).  Device memory: one book at a time plus the results.
 * Returns BT_OK, BT_EINVAL (bad arguments or no candidate could be built),
 * BT_ENOMEM or BT_EHIP.  A caller tuning a large batch can pass a sample of
 * it: the choice carries over to batches of the same mix. */
#define BT_AUTOTUNE_CANDIDATES 6
int bt_autotune(const bt_params *h_params, int32_t n, const bt_tune *base, const bt_tune *cand, int32_t n_cand,
                int32_t reps, void *stream, bt_tune *best, double *ms);

/* Plain single-option pricing: host in, host out, synchronous on the null
 * stream.  Uses a cached one-option book per calling thread, kept until
 * bt_shutdown on that thread. */
int bt_price(const bt_params *p, bt_result *out);

/* Frees what bt_price keeps between calls on the calling thread (its cached
 * one-option book and result buffer) and every workspace of bt_price_batch
 * and bt_price_grad_batch (of all threads; waits for each device first).
 * Books from bt_book_create are not affected, and later calls build new
 * caches.  Safe to call at any time, also repeatedly.  Returns BT_OK. */
int bt_shutdown(void);

/* Tree constants the library derives for one option on the host (u, d, r,
 * rho = 1/r, p = (r-d)/(u-d)); BT_EINVAL if the option is invalid. */
int bt_model_constants(const bt_params *p, double *u, double *d, double *r, double *rho, double *pu);

const char *bt_strerror(int code);
int bt_version(void);
int bt_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BT_H */
