"""Writes the algorithmic operation counts of the benchmark workload.

For every tree of the paper-scale grid (S0 = 100, K in {90, 100, 110},
R = 0.05, sigma = 0.3, T = 1, k in {0, .25, .5, 1} %, put and call, N = 1500
and N = 5000) the oracle counts the binary64 additions, subtractions,
multiplications and divisions of the canonical seller (ask) and buyer (bid)
recursions; the counts go to ``counts/paper_grid_flops.json``, where the
benchmark reads them to price the work of one launch.  Only the oracle is
called.

    python -m oracle.count_flops [threads]
"""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_1110_2477_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "counts", "paper_grid_flops.json")


def count(p):
    oracle.flops()
    oracle.price_params(p, sides=1)
    f_ask = oracle.flops()
    oracle.price_params(p, sides=2)
    f_bid = oracle.flops()
    return f_ask, f_bid


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    rows = []
    for N in (1500, 5000):
        g = W.paper_grid(N)
        order = sorted(range(len(g)), key=lambda i: -(g[i]["payoff"] * 10 + g[i]["k"]))
        with ThreadPoolExecutor(max_workers=threads) as ex:
            res = dict(zip(order, ex.map(lambda i: count(g[i]), order)))
        for i in range(len(g)):
            p = g[i]
            rows.append(dict(N=int(p["N"]), payoff=int(p["payoff"]), K=float(p["K"]), k=float(p["k"]),
                             ask_flops=int(res[i][0]), bid_flops=int(res[i][1])))
        print(f"N={N} done", flush=True)
    doc = {"workload": "paper_grid_put_call_N1500_N5000_48_trees",
           "counted_by": "oracle (binary64 add, sub, mul, div of the canonical recursion)",
           "trees": rows,
           "ask_flops": sum(r["ask_flops"] for r in rows),
           "bid_flops": sum(r["bid_flops"] for r in rows)}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(OUT, doc["ask_flops"], doc["bid_flops"])


if __name__ == "__main__":
    main()
