"""Writes paper_scale.json: the oracle's prices, breakpoint counts and (where
asked) tangents for the paper-scale parity cases of the GPU tests:

* the American put with N = 20000, S0 = K = 100, sigma = 0.4, T = 2,
  R = 0.05, k = 1 % (ask, bid, price0, counts);
* the 32 options of the Greeks book (N 500..1500) that the
  finite-difference check uses, with the oracle's forward-mode derivatives;
* a seeded 32-option sample of the stress book spanning N 64..8192, with 8
  costly calls and bull spreads at N >= 4000 (prices and counts).

Calls only ``oracle`` (the C oracle through its binding) and the input
generators of ``paper_1110_2477_amd.workloads``; takes about a quarter of an
hour on 8 cores.

    python tests/golden/make_paper_scale.py [threads]
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1110_2477_amd import workloads as W  # noqa: E402

FIELDS = ("S0", "K", "K2", "R", "sigma", "T", "k", "N", "payoff", "flags")


def record(p):
    return {f: (int(p[f]) if f in ("N", "payoff", "flags") else float(p[f])) for f in FIELDS}


def result(o):
    r = {k: (float(v) if isinstance(v, float) or hasattr(v, "dtype") and v.dtype.kind == "f" else v)
         for k, v in o.items() if not k.startswith("grad")}
    r = {k: (int(v) if k.startswith("bp_") else float(v)) for k, v in r.items()}
    for side in ("ask", "bid"):
        if "grad_" + side in o:
            r["grad_" + side] = [float(x) for x in o["grad_" + side]]
    return r


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    jobs = []   # (group, index in group, params, grad, sides)
    lp = W.long_put()[0]
    jobs.append(("long_put", 0, lp, False, 1))
    jobs.append(("long_put", 0, lp, False, 2))
    gb = W.greeks_book(1024, seed=4)
    for j, i in enumerate(W.greeks_fd_subset(len(gb))):
        jobs.append(("greeks_fd32", j, gb[i], True, 3))
    sb = W.stress_book(16384, seed=5)
    for j, i in enumerate(W.stress_sample(sb)):
        jobs.append(("stress_sample", j, sb[i], False, 3))
    order = sorted(range(len(jobs)), key=lambda q: -int(jobs[q][2]["N"]) * (5 if jobs[q][3] else 1))
    t0 = time.time()

    def run(q):
        g, j, p, grad, sides = jobs[q]
        t = time.time()
        o = oracle.price_params(p, grad=grad, sides=sides)
        print(f"{g}[{j}] N={int(p['N'])} payoff={int(p['payoff'])} k={float(p['k']):.4f}: "
              f"{time.time() - t:.1f} s", flush=True)
        return o

    with ThreadPoolExecutor(max_workers=threads) as ex:
        outs = dict(zip(order, ex.map(run, order)))
    groups = {"long_put": [], "greeks_fd32": [], "stress_sample": []}
    lp_res = {}
    for q, (g, j, p, grad, sides) in enumerate(jobs):
        o = outs[q]
        if g == "long_put":
            side = "ask" if sides == 1 else "bid"
            lp_res.update({side: float(o[side]), "price0": float(o["price0"]),
                           f"bp_total_{side}": int(o[f"bp_total_{side}"]),
                           f"bp_max_{side}": int(o[f"bp_max_{side}"])})
        else:
            groups[g].append(dict(params=record(p), oracle=result(o)))
    groups["long_put"] = [dict(params=record(lp), oracle=lp_res)]
    out = dict(source="tests/golden/make_paper_scale.py (oracle.price_params)",
               cite="Section 3 (seller's and buyer's recursions), Section 4.1 (tree), Appendix (zero-cost "
                    "price); inputs from paper_1110_2477_amd.workloads",
               seconds=time.time() - t0, **groups)
    with open(os.path.join(HERE, "paper_scale.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote paper_scale.json in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
