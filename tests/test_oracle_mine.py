"""Pins for the oracle's level-wise miner (Problem 1, Sec. 2) -- no GPU.

The mined sets are checked against exhaustive enumeration: every episode of
every size up to the level cap over the stream's alphabet and the interval
set is counted, and the frequent ones must be exactly what the miner
returns (so the candidate generation loses nothing and adds nothing)."""
import itertools

import numpy as np

import oracle
from oracle import mine
from paper_0905_2200_amd import synth


def _enumerate(n_types, N, intervals):
    for ty in itertools.product(range(n_types), repeat=N):
        for ivs in itertools.product(intervals, repeat=N - 1):
            yield (ty, tuple(l for l, _ in ivs), tuple(h for _, h in ivs))


def test_candidate_generation_by_hand():
    F1 = [0, 2]
    I = [(0, 5), (5, 9)]
    c2 = mine.gen_level2(F1, I)
    assert len(c2) == 2 * 2 * 2
    assert ((0, 0), (0,), (5,)) in c2 and ((2, 0), (5,), (9,)) in c2
    F2 = [((0, 1), (0,), (5,)), ((1, 2), (0,), (5,)), ((1, 2), (5,), (9,)), ((2, 1), (0,), (5,))]
    c3 = set(mine.gen_next(F2))
    want = {((0, 1, 2), (0, 0), (5, 5)), ((0, 1, 2), (0, 5), (5, 9)),
            ((1, 2, 1), (0, 0), (5, 5)), ((1, 2, 1), (5, 0), (9, 5)),
            ((2, 1, 2), (0, 0), (5, 5)), ((2, 1, 2), (0, 5), (5, 9))}
    assert c3 == want


def test_mined_sets_equal_exhaustive_enumeration():
    rng = np.random.default_rng(41)
    I = [(0, 3), (2, 6)]
    for trial in range(3):
        n_types = 3
        ids, ticks = synth.tiny_stream(rng, 300, n_types, 2)
        theta = int(rng.integers(12, 30))
        res = mine.mine(ids, ticks, n_types, I, theta, max_level=4, projection=False)
        for level in range(1, 5):
            eps = list(_enumerate(n_types, level, I))
            cnt = oracle.count_episodes(ids, ticks, eps, num_types=n_types)
            want = {e: int(c) for e, c in zip(eps, cnt) if c >= theta}
            got = res[level]["frequent"] if level in res else {}
            assert got == want, (trial, level, theta)


def test_mining_planted_cascade_found_and_anti_monotone():
    s = synth.config_mining(n_neurons=12, rate_hz=5.0, duration_s=60.0, n_cascades=2, tag=91)
    res = mine.mine(s["ids"], s["ticks"], s["num_types"], s["intervals"], s["theta"],
                    max_level=6)
    for c in s["cascades"]:
        if c["firings"] < s["theta"]:
            continue
        for L in range(2, len(c["neurons"]) + 1):
            for ep in synth.sub_episodes(c, L):
                assert ep in res[L]["frequent"], (ep, c["firings"])
    for level in res:
        if level < 3:
            continue
        prev = res[level - 1]["frequent"]
        for (ty, lo, hi), x in res[level]["frequent"].items():
            assert (ty[:-1], lo[:-1], hi[:-1]) in prev and (ty[1:], lo[1:], hi[1:]) in prev
            assert x <= prev[(ty[:-1], lo[:-1], hi[:-1])] and x <= prev[(ty[1:], lo[1:], hi[1:])]
        up, ex = res[level]["upper"], res[level]["exact"]
        assert ((ex == -1) | (up >= ex)).all()
