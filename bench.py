"""Benchmark: ask/bid/zero-cost pricing on one MI355X.

Workload (one step = one pass of the whole path over the workload): the
paper-scale grid of single American puts and calls, S0 = 100,
K in {90, 100, 110}, R = 0.05, sigma = 0.3, T = 1, k in {0, .25, .5, 1} %,
at N = 1500 and N = 5000 (48 trees), priced as one book: seller and buyer
recursions (ask, bid) and the zero-cost recursion (price0) of every tree.
Inputs are resident on the GPU before timing starts.

Printed: one JSON line with tree nodes/s (value), per-kernel HIP-event
times, the roofline of the dominant kernel (algorithmic and counter-based
figures, and the latency chain that binds it), batched options/s on the
mixed 4096-option book against plain single-option forward on the same
options, the Greeks book through the autograd Function, the stress mix (a
stated subset of its 16384 options in graph-captured batches, Greeks, and
the N = 20000 put), and the CPU oracle timed on the host on a bounded
sample, compared element by element with the GPU.

``--counter-summary DIR`` instead prints per-kernel means of the counters
in a rocprofv3 ``--pmc`` output directory (how profiles/ is written).
"""
import argparse
import csv
import glob
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
CLOCK_HZ = 2.4e9
N_CU = 256


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_leg(sample, cores):
    """Times the CPU oracle on a bounded sample: every option of the sample
    (ask, bid and price0), one option per task on `cores` threads; returns
    the timing and the oracle's results in sample order."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1110_2477_amd import workloads as W

    order = sorted(range(len(sample)), key=lambda i: -int(sample[i]["N"]))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        outs = list(ex.map(lambda i: oracle.price_params(sample[i]), order))
    dt = time.perf_counter() - t0
    res = [None] * len(sample)
    for i, o in zip(order, outs):
        res[i] = o
    nodes = W.nodes(sample)
    return dict(seconds=dt, nodes=nodes, nodes_per_s=nodes / dt, options_per_s=len(sample) / dt), res


def compare_with_oracle(gpu, ref):
    """Largest relative difference of ask, bid, price0 and whether every
    breakpoint count is equal, GPU results against oracle results."""
    worst, counts_equal, bitexact = 0.0, True, 0
    for r, o in zip(gpu, ref):
        for key in ("ask", "bid", "price0"):
            b = o[key]
            e = abs(r[key] - b) / abs(b) if b != 0 else abs(r[key])
            worst = max(worst, float(e))
        bitexact += int(r["ask"] == o["ask"] and r["bid"] == o["bid"] and r["price0"] == o["price0"])
        for key in ("bp_total_ask", "bp_total_bid", "bp_max_ask", "bp_max_bid"):
            counts_equal &= int(r[key]) == int(o[key])
    return dict(max_rel_err=worst, counts_equal=bool(counts_equal), bit_exact_options=bitexact, options=len(ref))


def kernel_source_digest():
    """SHA-256 over the HIP sources of the kernels with comments and blank
    space removed (the counters below are valid only for the code they were
    taken on; a change to a comment does not change the code)."""
    import hashlib
    import re

    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1110_2477_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(src, name), encoding="utf-8") as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            text = " ".join(text.split())
            h.update(name.encode() + b"\0" + text.encode())
    return h.hexdigest()


def _profile_kv(name):
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return kv


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading for
    a plain copy of known size), or None when the summary is missing or was
    taken on other kernel sources."""
    kv = _profile_kv("band_kernel_traffic_paper_grid.txt")
    if not kv or kv.get("kernel") != kernel:
        return None
    return float(kv["hbm_bytes_per_launch"])


def measured_counters(kernel):
    """Per-launch SQ counters of `kernel` from the committed summary
    (profiles/band_kernel_counters_paper_grid.txt), or None when missing or
    taken on other kernel sources."""
    kv = _profile_kv("band_kernel_counters_paper_grid.txt")
    if not kv:
        return None
    key = kernel.replace(" ", "")
    out = {k.split("|", 1)[1]: float(v) for k, v in kv.items() if k.startswith(key + "|")}
    return out or None


def counter_summary(d):
    """Per-kernel means of every counter in a rocprofv3 --pmc csv directory."""
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    acc = {}
    for r in rows:
        k = (r["Kernel_Name"], r["Counter_Name"])
        acc.setdefault(k, {})
        disp = r.get("Dispatch_Id") or r.get("Correlation_Id")
        acc[k][disp] = acc[k].get(disp, 0.0) + float(r["Counter_Value"])
    out = {}
    for (kern, ctr), per in sorted(acc.items()):
        vals = list(per.values())
        out.setdefault(kern, {})[ctr] = dict(dispatches=len(vals), mean=sum(vals) / len(vals))
    return out


def algorithm1_leg(bt, W, np, cores):
    """The paper's own parallel algorithm (Section 4.2, Algorithm 1) on the
    host's cores (libbtcpu): the paper's headline experiment -- the Table 2
    American put, N = 1500, k = 0.5 %, L = 5 -- serially and on 8 threads,
    and the grid's 24 N = 1500 trees one at a time on all cores."""
    put = W.book([dict(S0=100.0, K=100.0, R=0.1, sigma=0.2, T=0.25, k=0.005, N=1500, payoff=W.PUT)])[0]
    _, s1 = bt.cpu_price(put, 1, 5)
    _, s8 = bt.cpu_price(put, min(8, cores), 5)
    threads = min(64, cores)
    sample = W.paper_grid(1500)
    t = 0.0
    for p in sample:
        _, st = bt.cpu_price(p, threads, 5)
        t += st["seconds"]
    nodes = W.nodes(sample)
    return {"value": nodes / t, "unit": "tree nodes/s", "cores": threads, "kind": "paper_algorithm1",
            "sample": "the grid's 24 N=1500 trees (ask, bid, price0), one tree at a time on all threads, L = 5",
            "seconds": t,
            "table2_put_N1500": {"serial_ms": s1["seconds"] * 1e3, "threads": min(8, cores),
                                 "parallel_ms": s8["seconds"] * 1e3, "speedup": s1["seconds"] / s8["seconds"],
                                 "efficiency": s1["seconds"] / s8["seconds"] / min(8, cores),
                                 "paper": "5.26x, 65.75 % on 8 cores of 2x Xeon E5405 (serial 1983.7 ms)"}}


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


def plain_leg(bt, W, np, sample):
    """bt_price one option at a time (host in, host out, synchronous) over
    `sample`, after one untimed call per distinct N (bt_price rebuilds its
    cached one-option book when N changes, which is timed as part of the
    plain path)."""
    bt.bt_price(sample[0])
    t0 = time.perf_counter()
    res = [bt.bt_price(p) for p in sample]
    dt = time.perf_counter() - t0
    return dt, res


def stress_leg(bt, W, np, torch, n_batches):
    """The stress mix (16384 options, N log-uniform in [64, 8192]): its first
    n_batches batches of 2048 options as books replayed from captured HIP
    graphs with the autotuner's tuning, Greeks of its first 256 options
    through bt_price_grad_batch, and the N = 20000 put with and without
    Greeks.  Every job is timed whole (re-pricing of overflowed options
    included)."""
    res = {}
    stress = W.stress_book(16384, seed=5)
    pick = np.random.default_rng(66).choice(2048, 48, replace=False)
    log("stress: autotuning on 48 options of the first batch")
    t0 = time.perf_counter()
    best, _ = bt.bt_autotune(stress[:2048][np.sort(pick)], reps=1)
    tune = {k: best[k] for k in ("band_levels", "wgs_per_cu")}
    res["batch_tune"] = dict(tune, autotune_seconds=time.perf_counter() - t0)
    total_s, total_nodes, total_opts, repriced, ok = 0.0, 0, 0, 0, True
    per_batch = []
    for bi in range(n_batches):
        b = stress[2048 * bi:2048 * (bi + 1)]
        bk = bt.Book(b, tune=tune, graph=True)
        # one pass: the call captures the launch sequence and replays it
        dt, dt_call, n_over = timed_job(bk, False, torch, np, bt)
        ok &= bool(np.all(bk.results()["status"] == 0))
        bk.close()
        log(f"stress batch {bi}: {dt:.1f} s ({n_over} re-priced)")
        per_batch.append(dt * 1e3)
        total_s += dt
        total_nodes += W.nodes(b)
        total_opts += len(b)
        repriced += n_over
    res["forward_graph_batches"] = dict(
        options=total_opts, batches=n_batches, batch_size=2048, ms_per_batch=per_batch,
        options_per_s=total_opts / total_s, tree_nodes_per_s=total_nodes / total_s, ok=ok,
        options_repriced=repriced,
        subset=f"options 0..{total_opts - 1} of the 16384 (the first {n_batches} of 8 batches of 2048)")
    g = stress[:256]
    d = bt.params_tensor(g)
    # a call of the same size on short trees builds the workspace
    cheap = g.copy()
    cheap["N"] = 64
    log("stress: Greeks of 256 options")
    bt.price_batch(bt.params_tensor(cheap), max_N=8192, grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, gr = bt.price_batch(d, max_N=8192, grad=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = bt.as_results(out)
    res["greeks_batch_256"] = dict(options_per_s=len(g) / dt, ms=dt * 1e3, tree_nodes_per_s=W.nodes(g) / dt,
                                   ok=bool(np.all(r["status"] == 0)), entry="bt_price_grad_batch",
                                   subset="options 0..255 of the 16384")
    bt.bt_shutdown()
    log(f"stress: Greeks of 256 options {dt * 1e3:.0f} ms")
    lp = W.long_put()
    for greeks in (False, True):
        log(f"put N=20000, greeks={greeks}")
        bk = bt.Book(lp, greeks=greeks)
        (bk.price_grad if greeks else bk.price)()
        torch.cuda.synchronize()
        dt, _, _ = timed_job(bk, greeks, torch, np, bt)
        res["put_N20000_" + ("greeks" if greeks else "prices")] = dict(
            ms=dt * 1e3, tree_nodes_per_s=W.nodes(lp) / dt, ok=bool(np.all(bk.results()["status"] == 0)))
        bk.close()
    log(f"stress: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mixed-book, plain, Greeks-book and stress legs")
    ap.add_argument("--stress-batches", type=int, default=2, metavar="B",
                    help="batches of 2048 stress options timed in the stress leg (1..8; default 2)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB from one device buffer to another (the known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--counter-summary", metavar="DIR",
                    help="only print per-kernel means of the counters in a rocprofv3 --pmc output "
                         "directory (csv) and exit")
    args = ap.parse_args()
    if args.counter_summary:
        print(json.dumps(counter_summary(args.counter_summary), indent=1))
        return
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
    grid_res = book.results()
    assert remaining == 0 and np.all(grid_res["status"] == 0), grid_res["status"]
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
    crit_ms = None
    if not args.no_extra:
        # the latency chain: the grid's costliest tree (the N = 5000 call
        # with k = 1 %) priced alone; a step cannot end before its buyer
        # recursion
        crit = grid[(grid["N"] == 5000) & (grid["payoff"] == W.CALL) & (grid["K"] == 100.0) & (grid["k"] == 0.01)]
        cb = bt.Book(crit)
        cb.price()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cb.price()
        torch.cuda.synchronize()
        crit_ms = (time.perf_counter() - t0) * 1e3
        cb.close()
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
        # plain single-option forward against batched forward on the same
        # options: a seeded 32-option sample of the mixed book, priced one at
        # a time by bt_price, then as one book; the full book's rate above is
        # the batched figure at scale
        sp = np.sort(np.random.default_rng(34).choice(len(mixed), 32, replace=False))
        sample = mixed[sp]
        dt_plain, plain_res = plain_leg(bt, W, np, sample)
        sb = bt.Book(sample)
        sb.price()
        torch.cuda.synchronize()
        dt_b, _, _ = timed_job(sb, False, torch, np, bt)
        same = all(plain_res[i].tobytes() == sb.results()[i].tobytes() for i in range(len(sample)))
        sb.close()
        bt.bt_shutdown()
        extra["plain_vs_batched"] = dict(
            sample="32 options of the mixed 4096 book (numpy default_rng(34).choice)",
            plain_options_per_s=len(sample) / dt_plain, plain_tree_nodes_per_s=W.nodes(sample) / dt_plain,
            batched_same_options_per_s=len(sample) / dt_b,
            batched_full_book_options_per_s=extra["batched_mixed_4096"]["options_per_s"],
            batched_over_plain_same_options=dt_plain / dt_b,
            batched_full_book_over_plain=(len(mixed) / dt) / (len(sample) / dt_plain),
            same_results=bool(same))
        log(f"plain vs batched: {extra['plain_vs_batched']}")
        # batched forward + Greeks on the 1024-option Greeks book (N 500..1500)
        # through the autograd Function (bt_price_grad_batch on torch's
        # stream, parameters resident on the GPU), against the price-only
        # batch entry point on the same options
        from paper_1110_2477_amd.autograd import bt_autograd
        gb = W.greeks_book(1024, seed=4)
        spec = bt.params_tensor(gb)
        S0 = torch.tensor(gb["S0"], dtype=torch.float64, device="cuda", requires_grad=True)
        sig = torch.tensor(gb["sigma"], dtype=torch.float64, device="cuda", requires_grad=True)
        Rr = torch.tensor(gb["R"], dtype=torch.float64, device="cuda", requires_grad=True)
        kk = torch.tensor(gb["k"], dtype=torch.float64, device="cuda", requires_grad=True)

        def fwd_bwd():
            for t in (S0, sig, Rr, kk):
                t.grad = None
            ask, bid = bt_autograd(S0, sig, Rr, kk, spec, max_N=1500)
            (ask.sum() + bid.sum()).backward()
            return ask, bid

        log("greeks book: first call (builds the workspace)")
        fwd_bwd()
        torch.cuda.synchronize()
        log("greeks book: timed call")
        t0 = time.perf_counter()
        ask, bid = fwd_bwd()
        torch.cuda.synchronize()
        dt_g = time.perf_counter() - t0
        log(f"greeks book: {dt_g * 1e3:.1f} ms")
        ok = bool(torch.isfinite(ask).all().item() and torch.isfinite(bid).all().item())
        bt.price_batch(spec, max_N=1500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.price_batch(spec, max_N=1500)
        torch.cuda.synchronize()
        dt_p = time.perf_counter() - t0
        bt.bt_shutdown()
        # the same Greeks by the checkpointed reverse sweep
        # (bt_price_adjoint_batch) against forward mode on the first 64 puts
        # of the book: the reverse sweep recomputes every node with a
        # recording tape, so books whose nodes hold many points (calls and
        # spreads with costs) take it seconds per option.  Device memory of
        # each workspace from the free-memory difference around its first
        # call.
        sb_ = gb[gb["payoff"] == W.PUT][:64]
        sub = bt.params_tensor(sb_)
        cols = {name: torch.tensor(sb_[name], dtype=torch.float64, device="cuda", requires_grad=True)
                for name in ("S0", "sigma", "R", "k")}

        def sub_fwd_bwd(mode):
            for t in cols.values():
                t.grad = None
            a_, b_ = bt_autograd(cols["S0"], cols["sigma"], cols["R"], cols["k"], sub, max_N=1500, mode=mode)
            (a_.sum() + b_.sum()).backward()
            return a_, b_

        fa = {}
        for mode in ("forward", "adjoint"):
            log(f"greeks {mode} mode on 64 puts, through the autograd Function")
            torch.cuda.synchronize()
            free0, _ = torch.cuda.mem_get_info()
            sub_fwd_bwd(mode)
            torch.cuda.synchronize()
            free1, _ = torch.cuda.mem_get_info()
            t0 = time.perf_counter()
            a_, b_ = sub_fwd_bwd(mode)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            o_, g_ = bt.price_batch(sub, max_N=1500, grad=True, mode=mode)
            fa[mode] = dict(ms=ms, workspace_gib=(free0 - free1) / 2 ** 30, grads=bt.as_grads(g_),
                            ok=bool(np.all(bt.as_results(o_)["status"] == 0)
                                    and torch.isfinite(cols["S0"].grad).all().item()))
            bt.bt_shutdown()
        ga, gf = fa["adjoint"]["grads"], fa["forward"]["grads"]
        diff = max(float(np.max(np.abs(ga[k] - gf[k]) / np.maximum(1.0, np.abs(gf[k])))) for k in ga.dtype.names)
        extra["greeks_adjoint_vs_forward_64"] = dict(
            sample="the first 64 puts of the Greeks book (N 500..1500)", max_rel_diff=diff,
            adjoint=dict(options_per_s=64 / (fa["adjoint"]["ms"] * 1e-3), ms=fa["adjoint"]["ms"],
                         workspace_gib=fa["adjoint"]["workspace_gib"], ok=fa["adjoint"]["ok"],
                         entry="autograd Function (forward + backward) over bt_price_adjoint_batch "
                               "(reverse sweep, sqrt(N) checkpoints)"),
            forward=dict(options_per_s=64 / (fa["forward"]["ms"] * 1e-3), ms=fa["forward"]["ms"],
                         workspace_gib=fa["forward"]["workspace_gib"], ok=fa["forward"]["ok"],
                         entry="autograd Function (forward + backward) over bt_price_grad_batch "
                               "(tangents carried forward)"))
        log(f"adjoint vs forward: {extra['greeks_adjoint_vs_forward_64']}")
        extra["batched_greeks_1024"] = dict(options_per_s=len(gb) / dt_g, ms=dt_g * 1e3,
                                            price_only_ms=dt_p * 1e3, greeks_over_price=dt_g / dt_p,
                                            ok=ok, entry="autograd Function over bt_price_grad_batch "
                                                         "(forward + backward), price-only via bt_price_batch",
                                            plain_options_per_s=extra["plain_vs_batched"]["plain_options_per_s"])
        log(f"greeks book: {extra['batched_greeks_1024']}")
        extra["stress"] = stress_leg(bt, W, np, torch, max(1, min(8, args.stress_batches)))
    out.update(extra)

    # roofline of the dominant kernel.  achieved: binary64 operations of the
    # canonical algorithm for every tree of the workload (counted by the
    # oracle, stored by oracle/count_flops.py) per launch, over the kernel's
    # average launch time; one launch is one band of one party.  The counter
    # fields come from the committed rocprofv3 summary of the same sources.
    with open(os.path.join(ROOT, "oracle", "counts", "paper_grid_flops.json")) as f:
        counts = json.load(f)
    dom = max(("bid", "ask"), key=lambda k: kernel_ms[k])
    flops = counts[dom + "_flops"]
    n_launch = (int(grid["N"].max()) + 1 + 31) // 32
    ms_launch = kernel_ms[dom] / n_launch
    achieved = flops / n_launch / (ms_launch * 1e-3) / 1e12
    kernel = f"bt_band_kernel<{1 if dom == 'bid' else 0}, double>"
    roof = {"bound": "latency", "kernel": kernel,
            "achieved": achieved, "peak": PEAK_FP64_NONFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_NONFMA_TFLOPS, "traffic": measured_traffic(kernel),
            "flops_per_step": flops, "launches_per_step": n_launch,
            "flops_per_launch": flops / n_launch, "ms_per_launch": ms_launch,
            "binding": "the dependent chain of one tree's buyer recursion: each level waits for its "
                       "largest node, updated by its wavefront with a helper wave",
            "critical_tree_alone_ms": crit_ms, "step_over_critical_tree": ms_step / crit_ms if crit_ms else None}
    c = measured_counters(kernel)
    if c:
        f64 = sum(c.get(k, 0.0) for k in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                                           "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64"))
        simds = N_CU * 4
        # a wave64 vector instruction occupies a 16-lane SIMD for 4 cycles;
        # GRBM_GUI_ACTIVE is summed over the 8 XCDs and SQ_WAVE_CYCLES counts
        # in units of 4 cycles (both checked on bt_price0_kernel, whose
        # resident waves are known)
        roof["counters"] = {
            "fp64_valu_wave_insts_per_launch": f64,
            "fp64_valu_lane_ops_frac": f64 * 64 / (ms_launch * 1e-3) / (PEAK_FP64_NONFMA_TFLOPS * 1e12),
            "valu_wave_insts_per_launch": c.get("SQ_INSTS_VALU"),
            "valu_issue_frac": (c["SQ_INSTS_VALU"] * 4 / (ms_launch * 1e-3 * CLOCK_HZ * simds)
                                if c.get("SQ_INSTS_VALU") else None),
            "lds_wave_insts_per_launch": c.get("SQ_INSTS_LDS"),
            "lds_bank_conflict_per_access": (c["SQ_LDS_BANK_CONFLICT"] / max(1.0, c["SQ_LDS_IDX_ACTIVE"]
                                                                           - c["SQ_LDS_BANK_CONFLICT"])
                                             if c.get("SQ_LDS_IDX_ACTIVE") else None),
            "mean_resident_waves": (4 * c["SQ_WAVE_CYCLES"] / (c["GRBM_GUI_ACTIVE"] / 8)
                                    if c.get("SQ_WAVE_CYCLES") and c.get("GRBM_GUI_ACTIVE") else None),
            "wave_slots_at_this_occupancy": simds,
            "source": "profiles/band_kernel_counters_paper_grid.txt"}
    out["roofline"] = roof

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
        gpu_res = sb.results()
        sb.close()
        leg, ref = oracle_leg(sample, cores)
        out["cpu_baseline"] = {"value": leg["nodes_per_s"], "unit": "tree nodes/s", "cores": cores,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": "the 24 N=1500 trees of the grid and its 18 N=5000 trees other than "
                                         "the calls with k >= 0.5% (ask, bid, price0), one option per thread",
                               "options_per_s": leg["options_per_s"], "seconds": leg["seconds"],
                               "gpu_same_sample": {"value": W.nodes(sample) / gpu_sample_s,
                                                   "seconds": gpu_sample_s, "ok": sample_ok},
                               "gpu_vs_oracle": compare_with_oracle(gpu_res, ref)}
        out["cpu_baseline_algorithm1"] = algorithm1_leg(bt, W, np, cores)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
