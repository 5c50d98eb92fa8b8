"""Tuning never changes a result, and the autotuner picks among the
candidates it timed.

Band height (levels per launch, hence the width of the column blocks and of
their recomputed halos) and workgroups per CU change only how the work is cut
and scheduled, so prices, Greeks and breakpoint counts must be the same bytes
under every tuning, including band heights whose blocks split the large
nodes of a high-cost call differently."""
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
    b = W.random_small(40, seed=41, n_max=300)
    extra = W.book([
        dict(S0=100.0, K=100.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=700, payoff=W.CALL),
        dict(S0=100.0, K=95.0, K2=105.0, R=0.05, sigma=0.3, T=1.0, k=0.01, N=450, payoff=W.BULL),
        dict(S0=100.0, K=100.0, R=0.05, sigma=0.3, T=1.0, k=0.005, N=900, payoff=W.PUT),
    ])
    return np.concatenate([b, extra])


TUNINGS = [dict(band_levels=2), dict(band_levels=8, wgs_per_cu=1), dict(band_levels=17),
           dict(band_levels=32, wgs_per_cu=1), dict(band_levels=31, wgs_per_cu=2)]


def test_band_height_and_workgroups_do_not_change_results():
    b = _book()
    say(f"case: tune invariance, {len(b)} options, default vs {len(TUNINGS)} tunings")
    ref = bt.Book(b)
    ref.price()
    assert ref.resolve_overflow() == 0
    want = ref.results()
    ref.close()
    assert np.all(want["status"] == 0)
    for t in TUNINGS:
        say("tuning", t)
        bk = bt.Book(b, tune=t)
        bk.price()
        assert bk.resolve_overflow() == 0
        got = bk.results()
        bk.close()
        assert got.tobytes() == want.tobytes(), t


def test_band_height_does_not_change_greeks():
    b = _book()[-8:]
    say(f"case: tune invariance with Greeks, {len(b)} options, bands 32 and 5")
    outs = []
    for t in (dict(flags=bt.BT_TUNE_GREEKS), dict(flags=bt.BT_TUNE_GREEKS, band_levels=5)):
        bk = bt.Book(b, tune=t, greeks=True)
        bk.price_grad()
        assert bk.resolve_overflow(grad=True) == 0
        outs.append((bk.results().tobytes(), bk.grads().tobytes()))
        bk.close()
    assert outs[0] == outs[1]


def test_band_height_out_of_range_is_rejected():
    b = W.random_small(4, seed=42, n_max=50)
    say("case: band_levels 1 and 33 rejected")
    for band in (1, 33, -3):
        with pytest.raises(bt.BtError) as e:
            bt.Book(b, tune=dict(band_levels=band))
        assert e.value.code == bt.BT_EINVAL


def test_autotuner_returns_its_fastest_candidate():
    b = _book()
    say(f"case: autotuner, library list, {len(b)} options")
    best, timed = bt.bt_autotune(b, reps=1)
    assert len(timed) == bt.BT_AUTOTUNE_CANDIDATES
    ms = [m for _, m in timed]
    assert all(m > 0 for m in ms), timed
    fastest = timed[int(np.argmin(ms))][0]
    assert best["band_levels"] == fastest["band_levels"] and best["wgs_per_cu"] == fastest["wgs_per_cu"]
    say("case: autotuner, caller's list with a rejected candidate")
    cand = [dict(band_levels=40), dict(band_levels=16, wgs_per_cu=1), dict(band_levels=32)]
    best, timed = bt.bt_autotune(b, candidates=cand, reps=1)
    assert timed[0][1] == -1.0 and timed[1][1] > 0 and timed[2][1] > 0
    assert best["band_levels"] in (16, 32)
    # the tuned book prices the same bytes as the default one
    a = bt.Book(b)
    a.price()
    a.resolve_overflow()
    t = bt.Book(b, tune=best)
    t.price()
    t.resolve_overflow()
    assert a.results().tobytes() == t.results().tobytes()
    a.close()
    t.close()


def test_arena_sized_from_the_book_prices_high_cost_calls_in_one_pass():
    # a quarter of the mixed book: its high-cost call buyers grow nodes of
    # thousands of breakpoints, and all of them share one launch per band;
    # the book's arena is sized for them, so nothing overflows, and the
    # results are those of a book whose larger pools keep the big nodes out
    # of the arena
    b = W.mixed_book(4096, seed=3)[:1024]
    say(f"case: arena sizing, {len(b)} options of the mixed book")
    bk = bt.Book(b)
    bk.price()
    got = bk.results()
    bk.close()
    assert int(np.sum(got["status"] == bt.BT_EOVERFLOW)) == 0
    assert np.all(got["status"] == 0)
    say("case: arena sizing, reference with 4x pools")
    ref = bt.Book(b, tune=dict(pool_points=1 << 20))
    ref.price()
    assert ref.resolve_overflow() == 0
    want = ref.results()
    ref.close()
    assert got.tobytes() == want.tobytes()
