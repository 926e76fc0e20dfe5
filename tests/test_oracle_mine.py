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


def _as_tuples(t, a, b):
    return [(tuple(x), tuple(y), tuple(z)) for x, y, z in zip(t.tolist(), a.tolist(), b.tolist())]


def test_array_generation_equals_tuple_generation():
    """The array form of the candidate generation (used for the full-size
    golden values) yields the tuple form's candidates in the same order."""
    rng = np.random.default_rng(3)
    F1 = [0, 2, 5]
    I = [(0, 3), (2, 6), (1, 9)]
    assert _as_tuples(*mine.gen_level2_arrays(F1, I)) == mine.gen_level2(F1, I)
    checked = 0
    for trial in range(300):
        T = int(rng.integers(2, 5))
        Iv = I[:int(rng.integers(1, 4))]
        l = int(rng.integers(1, 5))
        eps = set()
        for _ in range(int(rng.integers(1, 60))):
            ty = tuple(int(x) for x in rng.integers(0, T, l))
            iv = [Iv[int(rng.integers(len(Iv)))] for _ in range(l - 1)]
            eps.add((ty, tuple(a for a, _ in iv), tuple(b for _, b in iv)))
        F = sorted(eps)
        t = np.array([e[0] for e in F], np.int32).reshape(len(F), l)
        a = np.array([e[1] for e in F], np.int32).reshape(len(F), l - 1)
        b = np.array([e[2] for e in F], np.int32).reshape(len(F), l - 1)
        assert _as_tuples(*mine.sort_episodes(t[::-1].copy(), a[::-1].copy(),
                                              b[::-1].copy())) == F
        got = _as_tuples(*mine.gen_next_arrays(t, a, b))
        assert got == mine.gen_next(F), trial
        checked += len(got)
    assert checked > 1000


def test_array_miner_equals_tuple_miner():
    for tr in range(2):
        s = synth.config_mining(n_neurons=10, rate_hz=15.0, duration_s=60.0, n_cascades=2,
                                tag=60 + tr)
        a = mine.mine_arrays(s["ids"], s["ticks"], s["num_types"], s["intervals"], s["theta"], 6,
                             keep=lambda L, M: True if L % 2 == 0 else np.arange(0, M, 7),
                             planted=lambda L: np.zeros((0, 3 * L - 2), np.int64))
        b = mine.mine(s["ids"], s["ticks"], s["num_types"], s["intervals"], s["theta"], 6)
        assert sorted(a) == sorted(b)
        for L in b:
            got = {e: (int(u), int(x)) for e, u, x in
                   zip(_as_tuples(a[L]["types"], a[L]["lo"], a[L]["hi"]), a[L]["upper"],
                       a[L]["exact"])}
            want = {e: (int(b[L]["upper"][k]), int(b[L]["exact"][k]))
                    for k, e in enumerate(b[L]["candidates"]) if e in b[L]["frequent"]}
            assert got == want, (tr, L)
            assert a[L]["n_candidates"] == len(b[L]["candidates"])
            if L > 1:
                assert a[L]["n_survivors"] == int((b[L]["upper"] >= s["theta"]).sum())
            if "all_types" in a[L]:
                assert _as_tuples(a[L]["all_types"], a[L]["all_lo"], a[L]["all_hi"]) == \
                    b[L]["candidates"]
                assert (a[L]["all_upper"] == b[L]["upper"]).all()
                kept = b[L]["exact"] >= 0
                assert (a[L]["all_exact"][kept] == b[L]["exact"][kept]).all()
                assert (a[L]["all_exact"] <= a[L]["all_upper"]).all()
            if "sample_idx" in a[L]:
                idx = a[L]["sample_idx"]
                assert _as_tuples(a[L]["sample_types"], a[L]["sample_lo"], a[L]["sample_hi"]) == \
                    [b[L]["candidates"][i] for i in idx]
                assert (a[L]["sample_upper"] == b[L]["upper"][idx]).all()
                kept = b[L]["exact"][idx] >= 0
                assert (a[L]["sample_exact"][kept] == b[L]["exact"][idx][kept]).all()
