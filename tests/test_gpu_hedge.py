"""Hedging output on the GPU (bt_book_price_hedge): the optimal stock
holdings at t = 0 of the seller and the buyer, equal to the oracle's bits
(oracle.hedge: the same minimisation, written independently, pinned to the
superhedging LP and the CRR delta in tests/test_oracle_hedge.py), for every
payoff shape and flag, small and paper-scale trees, and with prices equal to
bt_book_price's."""
import numpy as np
import pytest

import oracle
import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bt.lib()
    yield


@pytest.mark.parametrize("which", ["variants", "paper_grid_1500"])
def test_hedges_match_the_oracle(which):
    b = W.variants_book(70, seed=97, n_max=200) if which == "variants" else W.paper_grid(1500)
    say(f"case: hedges at t = 0, {which}, {len(b)} options")
    bk = bt.Book(b)
    bk.price_hedge()
    res, hg = bk.results(), bk.hedges()
    bk.price()
    assert bk.results().tobytes() == res.tobytes()
    bk.close()
    for i in range(len(b)):
        assert res[i]["status"] == 0
        o = oracle.hedge_params(b[i])
        got = (hg[i]["ask_lo"], hg[i]["ask_hi"], hg[i]["bid_lo"], hg[i]["bid_hi"])
        want = (o["ask"][0], o["ask"][1], o["bid"][0], o["bid"][1])
        assert got == want, (i, got, want, b[i])


def test_hedges_of_invalid_options_are_nan():
    b = W.single_put_n100().repeat(2)
    b[1]["sigma"] = -1.0
    bk = bt.Book(b)
    bk.price_hedge()
    hg = bk.hedges()
    bk.close()
    assert np.isfinite(hg[0]["ask_lo"]) and np.isnan(hg[1]["ask_lo"]) and np.isnan(hg[1]["bid_hi"])
