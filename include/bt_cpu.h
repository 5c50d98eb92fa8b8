/*
 * bt_cpu.h -- C ABI of libbtcpu: the paper's own parallel algorithm on the
 * host's cores, as a CPU baseline for the GPU library (bt.h).
 *
 * Zhang, Roux & Zastawniak (2011), Section 4.2 and Algorithm 1: the tree is
 * processed from level N+1 towards the root in rounds.  A round whose base
 * level B holds B+1 nodes gives each of the p threads floor((B+1)/p)
 * columns (the last thread the rest) and works D = min(L, floor((B+1)/p)-1)
 * levels down.  A thread first computes its region A, the nodes that need
 * nothing from another thread; it then waits for the signal of its right
 * neighbour, sent when that neighbour has finished the leftmost node of its
 * region A at level B-D+1 (B-D when D = 1), and computes its region B, the
 * triangle at its right edge.  All threads meet at the end of the round.
 * Whenever the next base level has fewer than 2p nodes, p drops by one
 * until it has at least two per thread.  Levels live in two buffers (seller
 * and buyer) of L+1 rows of N+2 records, level t in row t mod (L+1).
 * Readings where the printed algorithm is ambiguous: the number of nodes at
 * base level B is B+1 (so the split is floor((B+1)/p) and the drop test
 * B+1 < 2p), the drop test is applied before the first round too, and a
 * thread's count of processed nodes includes its leaves at level N+1; with
 * them the per-thread counts are those of the paper's Table 1.
 *
 * Every node is updated by the same per-node code as the GPU library
 * (bt_device.hpp, built for the host), so the prices and breakpoint counts
 * are the same bits.  The zero-cost price is the scalar recursion, run on
 * the calling thread.
 */
#ifndef BT_CPU_H
#define BT_CPU_H

#include <stdint.h>

#include "bt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Statistics of one bt_cpu_price call. */
typedef struct {
    double seconds;             /* wall time of the two recursions          */
    int64_t nodes[64];          /* nodes each thread computed (both parties
                                   count once), levels 0..N+1                */
    int32_t threads, rounds;    /* threads started, rounds run              */
} bt_cpu_stats;

/* Prices one option with Algorithm 1 on `threads` host threads (1..64) and
 * at most L levels per round (L >= 1).  p: host pointer to the option;
 * out: host pointer to its result (same fields and meaning as bt_result of
 * bt.h); stats: host pointer or NULL.  Synchronous.  Returns BT_OK,
 * BT_EINVAL (bad arguments: the option's status is BT_EINVAL when the
 * option itself is invalid and the call still returns BT_OK) or BT_ENOMEM. */
int bt_cpu_price(const bt_params *p, int32_t threads, int32_t L, bt_result *out, bt_cpu_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* BT_CPU_H */
