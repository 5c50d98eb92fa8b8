"""Batch entry points on device-resident options (bt_price_batch,
bt_price_grad_batch) and the autograd.Function built on them.

The batch path derives the trees and plans the band tasks on the GPU, then
runs the same kernels as a book: its results must be the book's bits
(book constants come from the host, batch constants from the device -- both
the correctly rounded exponentials), and therefore the oracle's."""
import sys

import numpy as np
import pytest

import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

from test_gpu_parity import check, say

pytestmark = pytest.mark.gpu

# sigma = exponent with T = N = 1: arguments whose libm exp is the other
# neighbour of e^x (the device must still match the host bit for bit)
HARD = ["0x1.a056d88f0ced3p-8", "0x1.88ab8b85f2710p-9", "0x1.983139ccee7acp-7", "0x1.6c15d3740474dp-9"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bt.lib()
    yield
    bt.bt_shutdown()


def _book_results(b, grad=False, tune=None):
    bk = bt.Book(b, tune=tune, greeks=grad)
    try:
        if grad:
            bk.price_grad()
            return bk.results(), bk.grads()
        bk.price()
        return bk.results()
    finally:
        bk.close()


def _mixed_with_edges():
    b = W.random_small(96, seed=71, n_max=160)
    hard = W.single_put_n100().repeat(len(HARD))
    for i, h in enumerate(HARD):
        hard[i]["sigma"], hard[i]["T"], hard[i]["N"], hard[i]["R"], hard[i]["k"] = float.fromhex(h), 1.0, 1, 0.0, 0.01
    bad = W.single_put_n100().repeat(3)
    bad[0]["N"] = 0          # invalid
    bad[1]["sigma"] = -0.2   # invalid
    bad[2]["N"] = 170        # above the call's max_N
    return np.concatenate([b, hard, bad])


def test_batch_matches_book_bits_and_oracle():
    import torch
    b = _mixed_with_edges()
    say(f"case: batch of {len(b)} (random small, hard exponents, invalid, N above max_N)")
    d = bt.params_tensor(b)
    out = bt.price_batch(d, max_N=160)
    torch.cuda.synchronize()
    r = bt.as_results(out)
    assert r[-3]["status"] == bt.BT_EINVAL and r[-2]["status"] == bt.BT_EINVAL and r[-1]["status"] == bt.BT_EINVAL
    assert np.isnan(r[-1]["ask"]) and r[-1]["bp_total_bid"] == 0
    ref = _book_results(b[:-3])
    assert r[:-3].tobytes() == ref.tobytes()
    check(b, r, range(len(b) - 3))


def test_batch_reuses_its_workspace_and_prices_smaller_calls():
    import torch
    b = W.mixed_book(64, seed=72, n_lo=100, n_hi=600)
    say("case: batch 64 options, then the first 17 with a smaller max_N")
    d = bt.params_tensor(b)
    r1 = bt.as_results(bt.price_batch(d, max_N=600))
    sub = b[:17]
    r2 = bt.as_results(bt.price_batch(bt.params_tensor(sub), max_N=int(sub["N"].max())))
    torch.cuda.synchronize()
    assert r1[:17].tobytes() == r2.tobytes()
    r3 = bt.as_results(bt.price_batch(d, max_N=600))
    assert r3.tobytes() == r1.tobytes()
    assert r1.tobytes() == _book_results(b).tobytes()


def test_grad_batch_matches_book_greeks_bits():
    import torch
    b = W.random_small(40, seed=73, n_max=120)
    say("case: grad batch of 40")
    out, g = bt.price_batch(bt.params_tensor(b), max_N=120, grad=True)
    torch.cuda.synchronize()
    r, gr = bt.as_results(out), bt.as_grads(g)
    rb, gb = _book_results(b, grad=True)
    assert r.tobytes() == rb.tobytes()
    assert gr.tobytes() == gb.tobytes()


def test_batch_captured_in_a_graph_replays_the_eager_bits():
    import torch
    b = W.mixed_book(48, seed=74, n_lo=64, n_hi=400)
    d = bt.params_tensor(b)
    say("case: batch captured in a torch CUDA graph, replayed 3 times")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        eager = bt.as_results(bt.price_batch(d, max_N=400, stream=s))   # builds the workspace
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # the workspace belongs to (device, stream): capture on the stream that
    # built it
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        out = bt.price_batch(d, max_N=400)
    ws_stream_out = None
    for rep in range(3):
        out.zero_()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = bt.as_results(out)
        assert got.tobytes() == eager.tobytes(), rep
        ws_stream_out = got
    assert ws_stream_out is not None


def test_batch_rejects_bad_arguments_and_empty_calls():
    import torch
    d = bt.params_tensor(W.single_put_n100())
    out = torch.empty(W.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    for max_N in (0, bt_max_n() + 1):
        with pytest.raises(bt.BtError) as e:
            bt.bt_price_batch(d.data_ptr(), 1, max_N, out.data_ptr())
        assert e.value.code == bt.BT_EINVAL
    bt.bt_price_batch(0, 0, 100, 0)   # n = 0: nothing to do
    with pytest.raises(bt.BtError):
        bt.bt_price_grad_batch(d.data_ptr(), 1, 100, out.data_ptr(), 0)


def bt_max_n():
    return 65536


def test_batch_overflow_gives_no_partial_result():
    import torch
    b = W.book([dict(S0=100.0, K=95.0, K2=105.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=400, payoff=W.BULL),
                dict(S0=100.0, K=100.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=600, payoff=W.CALL),
                dict(S0=100.0, K=100.0, R=0.05, sigma=0.3, T=1.0, k=0.005, N=300, payoff=W.PUT),
                # several breakpoints per node on average: more than one point
                # per node of band buffer
                dict(S0=100.0, K=100.0, R=0.03, sigma=0.15, T=0.5, k=0.08, N=500, payoff=W.CALL)])
    say("case: batch with level factor 1")
    r = bt.as_results(bt.price_batch(bt.params_tensor(b), max_N=600, tune=dict(level_factor=1)))
    torch.cuda.synchronize()
    n_over = 0
    for i in range(len(b)):
        assert r[i]["status"] in (0, bt.BT_EOVERFLOW)
        if r[i]["status"] == 0:
            check(b, r, [i])
        else:
            n_over += 1
            assert np.isnan(r[i]["ask"]) and np.isnan(r[i]["bid"]) and np.isnan(r[i]["price0"])
            assert r[i]["bp_total_ask"] == 0 and r[i]["bp_max_bid"] == 0
    say(f"  overflowed: {n_over}")
    assert n_over >= 1
    bt.bt_shutdown()   # the next tests build workspaces with the default tuning


def test_autograd_function_on_device_tensors():
    import torch
    from paper_1110_2477_amd.autograd import bt_autograd
    b = W.random_small(12, seed=75, n_max=90)
    b["flags"] = 0
    say("case: autograd on device tensors")
    dev = "cuda"
    S0 = torch.tensor(b["S0"], dtype=torch.float64, device=dev, requires_grad=True)
    sig = torch.tensor(b["sigma"], dtype=torch.float64, device=dev, requires_grad=True)
    R = torch.tensor(b["R"], dtype=torch.float64, device=dev, requires_grad=True)
    k = torch.tensor(b["k"], dtype=torch.float64, device=dev, requires_grad=True)
    ask, bid = bt_autograd(S0, sig, R, k, b)
    (ask.sum() + 2.0 * bid.sum()).backward()
    rb, gb = _book_results(b, grad=True)
    assert np.array_equal(ask.detach().cpu().numpy(), rb["ask"])
    assert np.array_equal(bid.detach().cpu().numpy(), rb["bid"])
    for t, name in ((S0, "dS0"), (sig, "dsigma"), (R, "dR"), (k, "dk")):
        want = gb["ask_" + name] + 2.0 * gb["bid_" + name]
        assert np.array_equal(t.grad.cpu().numpy(), want), name
    sys.stdout.flush()
