"""Exercise maps on the GPU (bt_book_price_exercise): for every node the byte
that says whether exercise attains the seller's and the buyer's expense at
zero stock holding, equal to the oracle's bytes (oracle.exercise: the same
decision taken on the oracle's own functions, pinned to the exact-rational
recursion and the zero-cost stopping region in
tests/test_oracle_exercise.py).  Every payoff shape and flag on small trees
(cooperative large-node path included), the paper grid at N = 1500 (trees
of several column blocks), prices equal to bt_book_price's, and 0xff planes
for an option that failed."""
from concurrent.futures import ThreadPoolExecutor

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
def test_exercise_maps_match_the_oracle(which):
    b = W.variants_book(70, seed=98, n_max=200) if which == "variants" else W.paper_grid(1500)
    say(f"case: exercise maps, {which}, {len(b)} options")
    bk = bt.Book(b)
    bk.price_exercise()
    res = bk.results()
    maps = [bk.exercise_maps(i) for i in range(len(b))]
    bk.price()
    assert bk.results().tobytes() == res.tobytes()
    bk.close()
    with ThreadPoolExecutor(max_workers=16) as ex:
        want = list(ex.map(lambda i: oracle.exercise_params(b[i]), range(len(b))))
    seen = 0
    for i in range(len(b)):
        assert res[i]["status"] == 0
        assert maps[i].shape == want[i].shape, i
        diff = np.nonzero(maps[i] != want[i])
        assert diff[0].size == 0, (i, b[i], diff[0][:3], diff[1][:3])
        seen += int(want[i].sum())
    assert seen > 0


def test_exercise_maps_of_a_failed_option_are_ff():
    b = W.single_put_n100().repeat(3)
    b[1]["sigma"] = -1.0
    b[2]["N"] = 7
    bk = bt.Book(b)
    bk.price_exercise()
    res = bk.results()
    m0, m1, m2 = (bk.exercise_maps(i) for i in range(3))
    bk.close()
    assert res[0]["status"] == 0 and res[1]["status"] == bt.BT_EINVAL and res[2]["status"] == 0
    assert m1.shape == (2, 101 * 102 // 2) and np.all(m1 == 0xFF)
    assert m2.shape == (2, 8 * 9 // 2)
    assert np.array_equal(m0, oracle.exercise_params(b[0]))
    assert np.array_equal(m2, oracle.exercise_params(b[2]))
