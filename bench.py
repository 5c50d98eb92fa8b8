"""Benchmark: ask/bid/zero-cost pricing on one MI355X.

Workload (one step = one pass of the whole path over the workload): the
paper-scale grid of single American puts and calls, S0 = 100,
K in {90, 100, 110}, R = 0.05, sigma = 0.3, T = 1, k in {0, .25, .5, 1} %,
at N = 1500 and N = 5000 (48 trees), priced as one book: seller and buyer
recursions (ask, bid) and the zero-cost recursion (price0) of every tree.
Inputs are resident on the GPU before timing starts.

Printed: one JSON line with tree nodes/s (value), per-kernel HIP-event
times, the roofline of the dominant kernel, batched options/s on a mixed
4096-option book, plain single-option forward on the same GPU, batched
prices with Greeks on a 1024-option book, and the CPU oracle timed on the
host on a bounded sample.
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
    """Times the CPU oracle on a bounded sample: every option of the sample
    (ask, bid and price0), one option per task on `cores` threads."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1110_2477_amd import workloads as W

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(oracle.price_params, sorted(sample, key=lambda p: -int(p["N"]))))
    dt = time.perf_counter() - t0
    nodes = W.nodes(sample)
    return dict(seconds=dt, nodes=nodes, nodes_per_s=nodes / dt, options_per_s=len(sample) / dt)


def kernel_source_digest():
    """SHA-256 over the HIP sources of the kernels (the counters below are
    valid only for the kernels they were taken on)."""
    import hashlib

    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1110_2477_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(src, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading for
    a plain copy of known size), or None when the summary is missing or was
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "band_kernel_traffic_paper_grid.txt")
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256") != kernel_source_digest() or kv.get("kernel") != kernel:
        return None
    return float(kv["hbm_bytes_per_launch"])


def timed_job(bk, greeks, torch, np, bt):
    """Times one whole pricing of a book: the pricing call, then the
    re-pricing of any option that outgrew its buffers.  Returns the total
    seconds, the seconds of the pricing call alone and the number of options
    re-priced."""
    call = bk.price_grad if greeks else bk.price
    t0 = time.perf_counter()
    call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_over = int(np.sum(bk.results()["status"] == bt.BT_EOVERFLOW))
    if n_over:
        bk.resolve_overflow(grad=greeks)
        torch.cuda.synchronize()
    return time.perf_counter() - t0, t1 - t0, n_over


def stress_leg(bt, W, np, torch):
    """One batch of 2048 options of the stress generator, and the long put."""
    res = {}
    batch = W.stress_book(16384, seed=5)[:2048]
    pick = np.random.default_rng(66).choice(len(batch), 256, replace=False)
    best, _ = bt.bt_autotune(batch[np.sort(pick)], reps=1)
    tune = {k: best[k] for k in ("band_levels", "wgs_per_cu")}
    for greeks in (False, True):
        # Greeks on the first 512 options of the batch (four times the work per option)
        b = batch[:512] if greeks else batch
        name = "batch_512_greeks" if greeks else "batch_2048_prices"
        bk = bt.Book(b, tune=tune, greeks=greeks, graph=True)
        call = bk.price_grad if greeks else bk.price
        log(f"{name}: capture and first call")
        call()
        torch.cuda.synchronize()
        log(f"{name}: timed call")
        dt, dt_call, n_over = timed_job(bk, greeks, torch, np, bt)
        log(f"{name}: {dt:.1f} s, of which {dt - dt_call:.1f} s re-pricing {n_over} options with larger levels")
        ok = bool(np.all(bk.results()["status"] == 0))
        bk.close()
        res[name] = dict(options_per_s=len(b) / dt, ms=dt * 1e3, tree_nodes_per_s=W.nodes(b) / dt, ok=ok,
                         pricing_call_ms=dt_call * 1e3, options_repriced=n_over)
        log(f"stress {name}: {res[name]}")
    res["batch_tune"] = tune
    lp = W.long_put()
    for greeks in (False, True):
        log(f"put N=20000, greeks={greeks}")
        bk = bt.Book(lp, greeks=greeks)
        call = bk.price_grad if greeks else bk.price
        call()
        torch.cuda.synchronize()
        dt, _, _ = timed_job(bk, greeks, torch, np, bt)
        res["put_N20000_" + ("greeks" if greeks else "prices")] = dict(ms=dt * 1e3, tree_nodes_per_s=W.nodes(lp) / dt,
                                                                    ok=bool(np.all(bk.results()["status"] == 0)))
        bk.close()
    log(f"stress: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed-book and plain legs")
    ap.add_argument("--stress", action="store_true",
                    help="also time the stress mix: one batch of 2048 options of the 16384-option "
                         "generator (N log-uniform in [64, 8192]) through a captured graph with the "
                         "autotuner's choice (prices; Greeks on its first 512), and the N=20000 put")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB from one device buffer to another (the known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n} bytes")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library prices a book on a single MI355X "
              "(options are independent, so a book would shard by option over several GPUs). "
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
    def step():
        # one complete pricing of the book: the kernels, then the host check
        # for options that outgrew the level buffers (re-priced with larger
        # ones inside the step when there are any)
        book.price()
        return book.resolve_overflow()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    book.timings()  # discard warm-up events
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    remaining = 0
    for _ in range(args.steps):
        remaining += step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, calls = book.timings()
    res = book.results()
    assert remaining == 0 and np.all(res["status"] == 0), res["status"]
    # how many options needed the second pass (same every step)
    book.price()
    n_resolved = int(np.sum(book.results()["status"] == bt.BT_EOVERFLOW))
    book.timings()
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
        "options_repriced_with_larger_levels_per_step": n_resolved,
    }

    extra = {}
    if not args.no_extra:
        mixed = W.mixed_book(4096, seed=3)
        mb = bt.Book(mixed, tune=dict(flags=bt.BT_TUNE_TIMING))
        mb.price()
        torch.cuda.synchronize()
        mb.timings()
        # whole job: the pricing call and the re-pricing of any option that
        # outgrew its buffers
        dt, dt_call, n_retry = timed_job(mb, False, torch, np, bt)
        mk, _ = mb.timings()
        r = mb.results()
        mb.close()
        extra["batched_mixed_4096"] = dict(options_per_s=len(mixed) / dt, tree_nodes_per_s=W.nodes(mixed) / dt,
                                           ms=dt * 1e3, pricing_call_ms=dt_call * 1e3, kernel_ms=mk,
                                           ok=bool(np.all(r["status"] == 0)), options_repriced=n_retry)
        log(f"mixed book: {extra['batched_mixed_4096']}")
        # the autotuner on a 512-option sample of the same mix, then the whole
        # book with its choice
        pick = np.random.default_rng(33).choice(len(mixed), 512, replace=False)
        t0 = time.perf_counter()
        best, timed = bt.bt_autotune(mixed[np.sort(pick)], reps=1)
        tune_s = time.perf_counter() - t0
        tb = bt.Book(mixed, tune=best)
        tb.price()
        torch.cuda.synchronize()
        dt_t, _, n_retry_t = timed_job(tb, False, torch, np, bt)
        tuned_ok = bool(np.all(tb.results()["status"] == 0)) and tb.results().tobytes() == r.tobytes()
        tb.close()
        extra["batched_mixed_4096_autotuned"] = dict(
            options_per_s=len(mixed) / dt_t, ms=dt_t * 1e3, same_results=tuned_ok, options_repriced=n_retry_t,
            tune={k: best[k] for k in ("band_levels", "wgs_per_cu")}, autotune_seconds=tune_s,
            candidates_ms_on_sample=[[c["band_levels"], c["wgs_per_cu"], m] for c, m in timed])
        log(f"autotuned mixed book: {extra['batched_mixed_4096_autotuned']}")
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
        # batched forward + Greeks (d ask, d bid / d S0, sigma, R, k) on the
        # 1024-option book with N in [500, 1500]
        gb = W.greeks_book(1024, seed=4)
        gk = bt.Book(gb, greeks=True)
        gk.price_grad()
        torch.cuda.synchronize()
        dt_g, _, n_retry = timed_job(gk, True, torch, np, bt)
        ok = bool(np.all(gk.results()["status"] == 0))
        t0 = time.perf_counter()
        gk.price()
        torch.cuda.synchronize()
        dt_p = time.perf_counter() - t0
        gk.close()
        extra["batched_greeks_1024"] = dict(options_per_s=len(gb) / dt_g, ms=dt_g * 1e3,
                                            price_only_ms=dt_p * 1e3, greeks_over_price=dt_g / dt_p,
                                            ok=ok, options_repriced=n_retry)
        log(f"greeks book: {extra['batched_greeks_1024']}")
    out.update(extra)

    # roofline of the dominant kernel: binary64 operations of the canonical
    # algorithm for every tree of the workload (counted by the oracle and
    # stored by oracle/count_flops.py) over the kernel's HIP-event time; one
    # launch is one band of one party, so flops / time over all launches is
    # the average flops per launch over the average launch duration
    with open(os.path.join(ROOT, "oracle", "counts", "paper_grid_flops.json")) as f:
        counts = json.load(f)
    dom = max(("bid", "ask"), key=lambda k: kernel_ms[k])
    flops = counts[dom + "_flops"]
    achieved = flops / (kernel_ms[dom] * 1e-3) / 1e12
    # one launch per band of the longest tree: bands of 32 levels over N+1 levels
    n_launch = (int(grid["N"].max()) + 1 + 31) // 32
    kernel = f"bt_band_kernel<{1 if dom == 'bid' else 0}, double>"
    out["roofline"] = {"bound": "alu", "kernel": kernel,
                       "achieved": achieved, "peak": PEAK_FP64_NONFMA_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_FP64_NONFMA_TFLOPS, "traffic": measured_traffic(kernel),
                       "flops_per_step": flops, "launches_per_step": n_launch,
                       "flops_per_launch": flops / n_launch,
                       "ms_per_launch": kernel_ms[dom] / n_launch}

    if args.stress:
        out["stress"] = stress_leg(bt, W, np, torch)

    cores = cpu_cores()
    if not args.no_cpu:
        g50 = W.paper_grid(5000)
        light = g50[(g50["k"] <= 0.0025) | (g50["payoff"] == 0)]
        sample = np.concatenate([W.paper_grid(1500), light])
        log(f"cpu oracle leg: {len(sample)} trees on {cores} threads")
        # the same sample on the GPU, one book, for a like-for-like ratio
        sb = bt.Book(sample)
        sb.price()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sb.price()
        torch.cuda.synchronize()
        gpu_sample_s = time.perf_counter() - t0
        sample_ok = sb.resolve_overflow() == 0 and bool(np.all(sb.results()["status"] == 0))
        sb.close()
        leg = oracle_leg(sample, cores)
        out["cpu_baseline"] = {"value": leg["nodes_per_s"], "unit": "tree nodes/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "the 24 N=1500 trees of the grid and its 18 N=5000 trees other than "
                                         "the calls with k >= 0.5% (ask, bid, price0), one option per thread",
                               "options_per_s": leg["options_per_s"], "seconds": leg["seconds"],
                               "gpu_same_sample": {"value": W.nodes(sample) / gpu_sample_s,
                                                   "seconds": gpu_sample_s, "ok": sample_ok}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
