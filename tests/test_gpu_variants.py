"""Every payoff shape through the GPU (delivered and cash-settled puts and
calls, bull and bear spreads, straddles; American, European and cost-at-t=0
variants) against the oracle: prices within 1e-10 with equal breakpoint
counts, through a book and through the batch entry point; Greeks, carried
forward and by the reverse sweep, within 1e-9 of the oracle's tangents."""
import numpy as np
import pytest

import oracle
import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

from test_gpu_greeks import grads_of
from test_gpu_parity import check, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bt.lib()
    yield
    bt.bt_shutdown()


def test_variants_book_and_batch_match_oracle():
    import torch
    b = W.variants_book(140, seed=95, n_max=220)
    say(f"case: {len(b)} options, every payoff shape and flag (book and batch)")
    res = bt.price_book(b)
    check(b, res)
    out = bt.price_batch(bt.params_tensor(b), max_N=220)
    torch.cuda.synchronize()
    assert bt.as_results(out).tobytes() == res.tobytes()


@pytest.mark.parametrize("mode", ["forward", "adjoint"])
def test_variants_greeks_match_oracle_tangents(mode):
    import torch
    b = W.variants_book(42, seed=96, n_max=120)
    say(f"case: Greeks ({mode}) of {len(b)} options of every payoff shape")
    out, g = bt.price_batch(bt.params_tensor(b), max_N=120, grad=True, mode=mode)
    torch.cuda.synchronize()
    res, g = bt.as_results(out), bt.as_grads(g)
    worst = 0.0
    for i in range(len(b)):
        o = oracle.price_params(b[i], grad=True)
        assert res[i]["status"] == 0
        assert res[i]["ask"] == o["ask"] and res[i]["bid"] == o["bid"], i
        for side in ("ask", "bid"):
            ad, ref = grads_of(g[i], side), o["grad_" + side]
            e = float(np.max(np.abs(ad - ref) / np.maximum(1.0, np.abs(ref))))
            worst = max(worst, e)
            assert e <= 1e-9, (i, side, ad, ref, b[i])
    say(f"  worst difference {worst:.3g}")
