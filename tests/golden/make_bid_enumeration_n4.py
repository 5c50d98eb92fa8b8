"""Writes bid_enumeration_n4.json: the buyer's price of two N = 4 options by
enumerating all 458,330 stopping times of the path tree, each priced by a
linear program (the definition of the bid in Section 3).  Calls only
``oracle.definitions``; takes a few minutes on 8 cores.

    python tests/golden/make_bid_enumeration_n4.py [workers]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import definitions as D  # noqa: E402

CASES = [
    # a call and a cash-settled bull spread: the buyers whose restriction is
    # the non-convex envelope
    dict(S0=100.0, K=100.0, K2=0.0, R=0.05, sigma=0.3, T=1.0, k=0.02, N=4, payoff=D.CALL),
    dict(S0=100.0, K=95.0, K2=105.0, R=0.1, sigma=0.2, T=0.25, k=0.01, N=4, payoff=D.BULL),
]


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    out = []
    for c in CASES:
        t0 = time.time()
        bid = D.bid_enum(c["S0"], c["K"], c["R"], c["sigma"], c["T"], c["k"], c["N"], payoff=c["payoff"],
                         K2=c["K2"], workers=workers)
        dt = time.time() - t0
        print(f"{c}: bid {bid!r} in {dt:.0f} s", flush=True)
        out.append(dict(c, bid_enumeration=bid, stopping_times=D.count_stopping_times(c["N"])))
    with open(os.path.join(HERE, "bid_enumeration_n4.json"), "w") as f:
        json.dump(dict(source="tests/golden/make_bid_enumeration_n4.py (oracle.definitions.bid_enum)",
                       cite="Section 3: the bid is the largest amount the buyer can borrow against "
                            "exercising at some stopping time; one LP per stopping time",
                       cases=out), f, indent=1)


if __name__ == "__main__":
    main()
