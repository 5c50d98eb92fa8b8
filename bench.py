"""Benchmark: ask/bid/zero-cost pricing on one MI355X.

Workload (one step = one pass of the whole path over the workload): the
paper-scale grid of single American puts and calls, S0 = 100,
K in {90, 100, 110}, R = 0.05, sigma = 0.3, T = 1, k in {0, .25, .5, 1} %,
at N = 1500 and N = 5000 (48 trees), priced as one book: seller and buyer
recursions (ask, bid) and the zero-cost recursion (price0) of every tree.
Inputs are resident on the GPU before timing starts.

Printed: one JSON line with tree nodes/s (value), per-kernel HIP-event
times, the roofline of the dominant kernel, batched options/s on a mixed
4096-option book, plain single-option forward on the same GPU, and the CPU
oracle timed on the host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and the FP64 vector rate for non-fused operations:
# 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 39.3 T binary64 add/mul/sub
# per second (the 78.6 TFLOP/s vector figure counts a fused multiply-add as
# two operations; this path performs no FMAs).
PEAK_FP64_NONFMA_TFLOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_leg(sample, cores):
    """Times the CPU oracle on a bounded sample: every option of the sample,
    one option per task on `cores` threads.  Also returns the algorithmic
    binary64 operation count per tree node of each side."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1110_2477_amd import workloads as W

    def one(p):
        oracle.flops()
        r_ask = oracle.price_params(p, sides=1)
        f_ask = oracle.flops()
        r_bid = oracle.price_params(p, sides=2)
        f_bid = oracle.flops()
        return f_ask, f_bid

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(one, sorted(sample, key=lambda p: -int(p["N"]))))
    dt = time.perf_counter() - t0
    nodes = W.nodes(sample)
    f_ask = sum(r[0] for r in res)
    f_bid = sum(r[1] for r in res)
    return dict(seconds=dt, nodes=nodes, nodes_per_s=nodes / dt, options_per_s=len(sample) / dt,
                flops_per_node_ask=f_ask / nodes, flops_per_node_bid=f_bid / nodes)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed-book and plain legs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build prices on a single MI355X "
              "(options are independent; see DESIGN.md for how a book would shard). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1110_2477_amd as bt
    from paper_1110_2477_amd import workloads as W

    torch.cuda.set_device(0)
    grid = np.concatenate([W.paper_grid(1500), W.paper_grid(5000)])
    nodes = W.nodes(grid)
    book = bt.Book(grid, tune=dict(flags=bt.BT_TUNE_TIMING))
    log(f"workload: 48-tree grid, {nodes} nodes; warmup {args.warmup}")
    for _ in range(args.warmup):
        book.price()
    torch.cuda.synchronize()
    book.timings()  # discard warm-up events
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        book.price()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, calls = book.timings()
    # options whose levels outgrow the buffers would need a second pass; the
    # timed calls are only valid if there were none
    assert book.resolve_overflow() == 0
    res = book.results()
    assert np.all(res["status"] == 0), res["status"]
    book.close()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = nodes * args.steps / (t1 - t0)
    kernel_ms = {k: v / calls for k, v in kms.items()}
    log(f"ms/step {ms_step:.3f}; kernels {kernel_ms}")

    out = {
        "metric": "tree nodes/s + batched options/s (ask,bid,Greeks) vs plain, at 1e-10 rel",
        "value": value,
        "unit": "tree nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "paper_grid_put_call_N1500_N5000_48_trees",
                   "options": int(len(grid)), "tree_nodes": nodes,
                   "N": [1500, 5000], "K": [90, 100, 110], "k": [0, 0.0025, 0.005, 0.01],
                   "S0": 100, "R": 0.05, "sigma": 0.3, "T": 1, "outputs": ["ask", "bid", "price0"]},
        "options_per_s": len(grid) * args.steps / (t1 - t0),
        "kernel_ms": kernel_ms,
    }

    extra = {}
    if not args.no_extra:
        mixed = W.mixed_book(4096, seed=3)
        mb = bt.Book(mixed, tune=dict(flags=bt.BT_TUNE_TIMING))
        mb.price()
        torch.cuda.synchronize()
        mb.timings()
        t0 = time.perf_counter()
        mb.price()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mk, _ = mb.timings()
        n_retry = int(np.sum(mb.results()["status"] == bt.BT_EOVERFLOW))
        mb.resolve_overflow()
        r = mb.results()
        mb.close()
        extra["batched_mixed_4096"] = dict(options_per_s=len(mixed) / dt, tree_nodes_per_s=W.nodes(mixed) / dt,
                                           ms=dt * 1e3, kernel_ms=mk, ok=bool(np.all(r["status"] == 0)),
                                           options_needing_larger_levels=n_retry)
        log(f"mixed book: {extra['batched_mixed_4096']}")
        # plain single-option forward: bt_price per option, synchronous
        sub = grid[[0, 5, 11, 18]]  # four N=1500 trees (put and call, several k)
        bt.bt_price(sub[0])
        t0 = time.perf_counter()
        for p in sub:
            bt.bt_price(p)
        dt = time.perf_counter() - t0
        extra["plain_single_option_forward"] = dict(options_per_s=len(sub) / dt,
                                                    tree_nodes_per_s=W.nodes(sub) / dt,
                                                    sample="4 N=1500 trees of the grid, bt_price one at a time")
        log(f"plain: {extra['plain_single_option_forward']}")
    out.update(extra)

    # roofline of the dominant kernel: binary64 operations of the canonical
    # algorithm per node (counted by the oracle on the sample below) x nodes
    # of one launch, over the kernel's HIP-event duration
    cores = cpu_cores()
    if not args.no_cpu:
        sample = W.paper_grid(1500)
        log(f"cpu oracle leg: 24 N=1500 trees on {cores} threads")
        leg = oracle_leg(sample, cores)
        out["cpu_baseline"] = {"value": leg["nodes_per_s"], "unit": "tree nodes/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "the 24 N=1500 trees of the grid (ask, bid, price0), one option "
                                         "per thread; N=5000 half not run",
                               "options_per_s": leg["options_per_s"], "seconds": leg["seconds"]}
        dom = max(("bid", "ask"), key=lambda k: kernel_ms[k])
        fpn = leg["flops_per_node_" + dom]
        flops = fpn * nodes
        achieved = flops / (kernel_ms[dom] * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": f"bt_item_kernel<{dom}>",
                           "achieved": achieved, "peak": PEAK_FP64_NONFMA_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / PEAK_FP64_NONFMA_TFLOPS, "traffic": None,
                           "flops_per_node": fpn, "flops_per_launch": flops}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
