"""The paper's Algorithm 1 on host threads (libbtcpu, include/bt_cpu.h):
prices and breakpoint counts equal the oracle's bits for every payoff shape
and flag, thread count and round height; and the nodes each thread computes
are the paper's Table 1 counts (tests/golden/table1_node_counts.json)."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_node_counts.json")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_1110_2477_amd import build as B
    if not os.path.exists(B.CPU_LIB):
        B.build_cpu()
    bt.cpu_lib()


def _same(r, o):
    assert r["status"] == 0
    assert r["ask"] == o["ask"] and r["bid"] == o["bid"] and r["price0"] == o["price0"]
    for key in ("bp_total_ask", "bp_total_bid", "bp_max_ask", "bp_max_bid"):
        assert int(r[key]) == o[key], key


@pytest.mark.parametrize("threads,L", [(1, 5), (2, 1), (3, 5), (8, 3), (5, 32)])
def test_prices_match_the_oracle(threads, L):
    b = np.concatenate([W.random_small(12, seed=200 + threads, n_max=90),
                        W.variants_book(14, seed=300 + threads, n_max=90)])
    for p in b:
        r, st = bt.cpu_price(p, threads, L)
        _same(r, oracle.price_params(p))
        N = int(p["N"])
        assert sum(st["nodes"]) == (N + 2) * (N + 3) // 2   # levels 0..N+1, each node once


def test_tiny_trees_drop_threads():
    for N in (1, 2, 3, 7):
        p = W.book([dict(S0=100.0, K=100.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=N, payoff=W.CALL)])[0]
        r, st = bt.cpu_price(p, 8, 5)
        _same(r, oracle.price_params(p))


def test_thread_zero_counts_are_table_1():
    with open(GOLDEN) as f:
        g = json.load(f)
    for ps, row in g["counts"].items():
        for Ns, want in row.items():
            p = W.book([dict(S0=100.0, K=100.0, R=0.1, sigma=0.2, T=0.25, k=0.005, N=int(Ns), payoff=W.PUT)])[0]
            r, st = bt.cpu_price(p, int(ps), g["L"])
            assert st["nodes"][0] == want, (ps, Ns, st["nodes"][0], want)
    # and the answer does not depend on the partition
    r1, _ = bt.cpu_price(p, 1, 5)
    _same(r, dict(ask=r1["ask"], bid=r1["bid"], price0=r1["price0"], bp_total_ask=int(r1["bp_total_ask"]),
                  bp_total_bid=int(r1["bp_total_bid"]), bp_max_ask=int(r1["bp_max_ask"]),
                  bp_max_bid=int(r1["bp_max_bid"])))


def test_bad_arguments():
    p = W.single_put_n100()[0]
    for threads, L in ((0, 5), (65, 5), (2, 0)):
        with pytest.raises(bt.BtError):
            bt.cpu_price(p, threads, L)
    q = p.copy()
    q["N"] = 0
    r, _ = bt.cpu_price(q, 2, 5)
    assert r["status"] == bt.BT_EINVAL and np.isnan(r["ask"])
