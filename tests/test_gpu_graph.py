"""Graph replay (BT_TUNE_GRAPH): every replay of a book's captured launch
sequence gives the same bytes as direct launches, with other GPU work and
synchronisations between the replays, for prices and for Greeks."""
import sys

import numpy as np
import pytest

import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _book():
    b = W.random_small(48, seed=31, n_max=250)
    extra = W.book([
        dict(S0=100.0, K=100.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=600, payoff=W.CALL),
        dict(S0=100.0, K=90.0, K2=99.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=500, payoff=W.BULL),
    ])
    return np.concatenate([b, extra])


def test_graph_replays_match_direct_launches():
    import torch
    b = _book()
    say("case: graph replay, 50 options, 3 replays with other work between")
    direct = bt.Book(b)
    direct.price()
    want = direct.results()
    other = bt.Book(W.random_small(16, seed=32, n_max=120))
    g = bt.Book(b, graph=True)
    for rep in range(3):
        g.price()
        got = g.results()
        assert got.tobytes() == want.tobytes(), rep
        # unrelated eager work and a synchronisation between replays
        other.price()
        x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
        float(x.sum().item())
        torch.cuda.synchronize()
    # a new output buffer is a new capture
    g.out = torch.empty_like(g.out)
    g.price()
    assert g.results().tobytes() == want.tobytes()
    for bk in (direct, other, g):
        bk.close()


def test_graph_replays_match_for_greeks():
    b = _book()[:20]
    say("case: graph replay with Greeks, 20 options, 2 replays")
    direct = bt.Book(b, greeks=True)
    direct.price_grad()
    want_r, want_g = direct.results(), direct.grads()
    g = bt.Book(b, greeks=True, graph=True)
    for rep in range(2):
        g.price_grad()
        assert g.results().tobytes() == want_r.tobytes(), rep
        assert g.grads().tobytes() == want_g.tobytes(), rep
        direct.price()
    direct.close()
    g.close()
