"""The no-allocation entry point (bt_price_batch_static) against the batch
entry point it varies (bt_price_batch), through the C ABI: the same bits on
two calls in a row, the second with a smaller input, and its limits."""
import numpy as np
import pytest

import paper_1110_2477_amd as bt
from paper_1110_2477_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bt.lib()
    yield


def _static(b, max_N):
    import torch
    d = bt.params_tensor(b)
    out = torch.full((len(b) * W.RESULT_DTYPE.itemsize,), 0xAB, dtype=torch.uint8, device="cuda")
    bt.bt_price_batch_static(d.data_ptr(), len(b), max_N, out.data_ptr())
    torch.cuda.synchronize()
    return bt.as_results(out)


def _batch(b, max_N):
    import torch
    r = bt.as_results(bt.price_batch(bt.params_tensor(b), max_N=max_N))
    torch.cuda.synchronize()
    return r


def test_static_matches_batch_on_two_calls_the_second_smaller():
    b1 = W.mixed_book(bt.BT_STATIC_MAX_OPTIONS, seed=81, n_lo=200, n_hi=600)
    b1[5]["N"] = bt.BT_STATIC_MAX_N   # the largest tree the entry point takes
    b1[3]["N"] = 0   # an invalid option
    say(f"case: static entry, {len(b1)} options, N 200..600 and one {bt.BT_STATIC_MAX_N}")
    s1 = _static(b1, bt.BT_STATIC_MAX_N)
    r1 = _batch(b1, bt.BT_STATIC_MAX_N)
    ok = s1["status"] == 0
    say(f"  BT_OK {int(ok.sum())}/{len(b1)}, statuses {sorted(set(s1['status'].tolist()))}")
    assert s1[3]["status"] == bt.BT_EINVAL
    # every option priced by both entry points has the same bits; one that
    # outgrew the smaller static buffers says so and carries no result
    both = ok & (r1["status"] == 0)
    assert both.sum() >= len(b1) - 4
    assert s1[both].tobytes() == r1[both].tobytes()
    over = s1["status"] == bt.BT_EOVERFLOW
    assert np.all(np.isnan(s1[over]["ask"])) and np.all(s1[over]["bp_total_bid"] == 0)

    b2 = W.random_small(21, seed=82, n_max=150)
    say(f"case: static entry again, {len(b2)} options, N up to 150")
    s2 = _static(b2, 150)
    r2 = _batch(b2, 150)
    assert np.all(s2["status"] == 0)
    assert s2.tobytes() == r2.tobytes()


def test_static_rejects_sizes_beyond_its_limits():
    import torch
    b = W.single_put_n100().repeat(bt.BT_STATIC_MAX_OPTIONS + 1)
    d = bt.params_tensor(b)
    out = torch.empty(len(b) * W.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    for n, max_N in ((len(b), 100), (1, bt.BT_STATIC_MAX_N + 1), (1, 0)):
        with pytest.raises(bt.BtError) as e:
            bt.bt_price_batch_static(d.data_ptr(), n, max_N, out.data_ptr())
        assert e.value.code == bt.BT_EINVAL
