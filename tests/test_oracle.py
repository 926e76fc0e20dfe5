"""Pins for the CPU oracle (no GPU).

Each test ties the oracle's Algorithm 1 / Algorithm 3 / Algorithm 4 counters
to something other than themselves: brute force from the Sec. 2 definition,
planted cascades whose count is known by construction, the paper's Theorem
and Observation (Sec. 5.3), closed forms and metamorphic properties.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_0905_2200_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
EXACT, RELAXED, RLISTS = oracle.MODE_EXACT, oracle.MODE_RELAXED, oracle.MODE_RELAXED_LISTS


def _all_episodes(n_types, N, intervals):
    out = []
    for ty in itertools.product(range(n_types), repeat=N):
        for ivs in itertools.product(intervals, repeat=N - 1):
            out.append((ty, tuple(l for l, _ in ivs), tuple(h for _, h in ivs)))
    return out


def _counts(ids, ticks, eps, mode, n_types):
    return oracle.count_episodes(ids, ticks, eps, mode=mode, num_types=n_types, nthreads=1)


# ---------------------------------------------------------------- P9 golden
def test_golden_sec2_examples():
    g = json.load(open(os.path.join(HERE, "golden", "paper_sec2_examples.json")))
    for c in g["cases"]:
        e = c["episode"]
        ep = [(tuple(e["types"]), tuple(e["lo"]), tuple(e["hi"]))]
        occ = brute.occurrences(c["ids"], c["ticks"], e["types"], e["lo"], e["hi"])
        assert len(occ) == c["occurrences"]
        assert brute.max_disjoint_exhaustive(occ) == c["count"]
        assert _counts(c["ids"], c["ticks"], ep, EXACT, 3)[0] == c["count"]
        if "relaxed_count" in c:
            assert _counts(c["ids"], c["ticks"], ep, RELAXED, 3)[0] == c["relaxed_count"]


# ---------------------------------------------------------------- P1 brute force
def test_brute_force_methods_agree():
    rng = np.random.default_rng(7)
    for _ in range(300):
        ids, ticks = synth.tiny_stream(rng, int(rng.integers(1, 11)), 2, 3)
        for ep in _all_episodes(2, 2, [(0, 2), (1, 3)]):
            occ = brute.occurrences(ids, ticks, *ep)
            assert brute.max_disjoint_dp(occ) == brute.max_disjoint_exhaustive(occ)


INTERVALS_TINY = [(0, 1), (0, 2), (1, 3), (2, 4)]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_exhaustive_tiny_streams(n):
    """Every stream of length n over 2 types with ticks 0..3 (ties in every
    order), every episode of 1-3 nodes over the tiny interval set."""
    eps = (_all_episodes(2, 1, []) + _all_episodes(2, 2, INTERVALS_TINY) +
           _all_episodes(2, 3, INTERVALS_TINY[:3]))
    for ids, ticks in brute.all_streams(n, 2, 3):
        ex = _counts(ids, ticks, eps, EXACT, 2)
        rx = _counts(ids, ticks, eps, RELAXED, 2)
        for k, ep in enumerate(eps):
            assert ex[k] == brute.count(ids, ticks, *ep), (ids, ticks, ep)
            assert rx[k] == brute.count(ids, ticks, *ep, relaxed=True), (ids, ticks, ep)


def test_random_tiny_streams():
    rng = np.random.default_rng(2024)
    eps = _all_episodes(3, 2, [(0, 2), (1, 4)]) + _all_episodes(3, 3, [(0, 3), (1, 4)])[::3] \
        + _all_episodes(2, 4, [(0, 3), (1, 5)])[::5]
    for trial in range(4000):
        n = int(rng.integers(0, 15))
        ids, ticks = synth.tiny_stream(rng, n, 3, 3)
        ex = _counts(ids, ticks, eps, EXACT, 3)
        rx = _counts(ids, ticks, eps, RELAXED, 3)
        for k, ep in enumerate(eps):
            assert ex[k] == brute.count(ids, ticks, *ep), (trial, ep)
            assert rx[k] == brute.count(ids, ticks, *ep, relaxed=True), (trial, ep)


@pytest.mark.slow
def test_random_tiny_streams_many_seeds():
    rng = np.random.default_rng(99)
    eps = _all_episodes(3, 2, [(0, 2), (1, 4)]) + _all_episodes(3, 3, [(0, 3), (2, 5)])
    for trial in range(100_000):
        ids, ticks = synth.tiny_stream(rng, int(rng.integers(0, 13)), 3, 4)
        ex = _counts(ids, ticks, eps, EXACT, 3)
        rx = _counts(ids, ticks, eps, RELAXED, 3)
        for k, ep in enumerate(eps):
            assert ex[k] == brute.count(ids, ticks, *ep)
            assert rx[k] == brute.count(ids, ticks, *ep, relaxed=True)


# ---------------------------------------------------------------- P2 planted cascades
def test_planted_clean_cascades():
    """Cascade neurons fire only inside the cascade and firings are more
    than the span apart: every contiguous sub-episode with the planted
    intervals counts exactly the number of firings, in both passes."""
    rng = np.random.default_rng(5)
    for trial in range(6):
        L = int(rng.integers(2, 8))
        ivs = [synth.INTERVALS[int(rng.integers(3))] for _ in range(L - 1)]
        neurons = list(range(L))
        dur = 600_000
        ci, ct, on = synth.cascade_firings(rng, neurons, ivs, dur, n_firings=150)
        bg_rates = np.zeros(30)
        bg_rates[L:] = 20.0
        bi, bt = synth.background(rng, bg_rates, dur)
        ids, ticks = synth.sort_events(np.concatenate([ci, bi]), np.concatenate([ct, bt]))
        casc = {"neurons": neurons, "intervals": ivs}
        for k in range(1, L + 1):
            eps = synth.sub_episodes(casc, k)
            ex = _counts(ids, ticks, eps, EXACT, 30)
            rx = _counts(ids, ticks, eps, RELAXED, 30)
            assert (ex == on.size).all() and (rx == on.size).all(), (trial, k, ex, rx, on.size)


def test_planted_cascades_with_background_lower_bound():
    s = synth.config_plain()
    for c in s["cascades"]:
        for k in (2, 3, 4):
            eps = synth.sub_episodes(c, k)
            ex = _counts(s["ids"], s["ticks"], eps, EXACT, 64)
            assert (ex >= c["firings"]).all()


# ---------------------------------------------------------------- P3, P4, P5
def _random_eps(rng, M, n_types, nmax):
    return synth.random_episodes(rng, M, n_types, nmax, synth.INTERVALS, n_min=1)


def test_theorem_upper_bound_and_observation():
    rng = np.random.default_rng(11)
    ids, ticks = synth.background(rng, np.full(8, 40.0), 100_000)
    ids, ticks = synth.sort_events(ids, ticks)
    eps = _random_eps(rng, 400, 8, 5)
    ex = _counts(ids, ticks, eps, EXACT, 8)
    rx = _counts(ids, ticks, eps, RELAXED, 8)
    rl = _counts(ids, ticks, eps, RLISTS, 8)
    assert (rx >= ex).all()          # Theorem of Sec. 5.3.2
    assert (rx == rl).all()          # Observation of Sec. 5.3.1
    assert ex.sum() > 0


def test_special_case_lo0_no_ties_a1_equals_a2():
    rng = np.random.default_rng(3)
    ids, ticks = synth.background(rng, np.full(6, 30.0), 200_000)
    ids, ticks = synth.sort_events(ids, ticks)
    # make ticks strictly increasing so no two events share a tick
    ticks = (ticks.astype(np.int64) * 4 + np.arange(ticks.size) % 4).astype(np.int32)
    order = np.argsort(ticks, kind="stable")
    ids, ticks = ids[order], ticks[order]
    assert (np.diff(ticks) > 0).all()
    eps = [(e[0], tuple(0 for _ in e[1]), e[2]) for e in _random_eps(rng, 200, 6, 5)]
    assert (_counts(ids, ticks, eps, EXACT, 6) == _counts(ids, ticks, eps, RELAXED, 6)).all()


# ---------------------------------------------------------------- P6 closed forms
def test_single_node_is_histogram():
    s = synth.config_plain()
    eps = [((e,), (), ()) for e in range(64)]
    hist = np.bincount(s["ids"], minlength=64)
    assert (_counts(s["ids"], s["ticks"], eps, EXACT, 64) == hist).all()
    assert (_counts(s["ids"], s["ticks"], eps, RELAXED, 64) == hist).all()


def test_hi_below_min_gap_gives_zero():
    ids = np.array([0, 1, 0, 1, 2], np.int32)
    ticks = np.array([0, 10, 20, 30, 40], np.int32)
    eps = [((0, 1), (0,), (9,)), ((1, 2), (0,), (9,)), ((0, 1, 2), (0, 0), (9, 100))]
    assert (_counts(ids, ticks, eps, EXACT, 3) == 0).all()
    assert (_counts(ids, ticks, eps, RELAXED, 3) == 0).all()


def test_closed_form_alternating():
    """A B A B ... with gap g: A->B (lo,hi] counts every pair iff lo<g<=hi."""
    k = 500
    ids = np.tile([0, 1], k).astype(np.int32)
    for g in (1, 7, 50):
        ticks = (np.arange(2 * k) * g).astype(np.int32)
        for lo, hi in ((0, 50), (g - 1, g), (g, g + 5), (0, g - 1)):
            if hi <= lo or hi < 0:
                continue
            if lo < g <= hi:
                want = k          # adjacent pairs, one per B
            elif any(lo < (2 * j + 1) * g <= hi for j in range(2 * k)):
                continue          # only non-adjacent pairs qualify: no simple closed form
            else:
                want = 0
            assert _counts(ids, ticks, [((0, 1), (lo,), (hi,))], EXACT, 2)[0] == want


# ---------------------------------------------------------------- P7 monotonicity
def test_monotonicity():
    rng = np.random.default_rng(17)
    ids, ticks = synth.background(rng, np.full(6, 40.0), 80_000)
    ids, ticks = synth.sort_events(ids, ticks)
    eps = _random_eps(rng, 150, 6, 4)
    eps = [e for e in eps if len(e[0]) >= 2]
    base = _counts(ids, ticks, eps, EXACT, 6)
    wider = [(ty, tuple(max(0, l - 7) for l in lo), tuple(h + 13 for h in hi)) for ty, lo, hi in eps]
    assert (_counts(ids, ticks, wider, EXACT, 6) >= base).all()
    keep = rng.random(ids.size) > 0.2
    assert (_counts(ids[keep], ticks[keep], eps, EXACT, 6) <= base).all()
    pre = [(ty[:-1], lo[:-1], hi[:-1]) for ty, lo, hi in eps]
    suf = [(ty[1:], lo[1:], hi[1:]) for ty, lo, hi in eps]
    assert (base <= _counts(ids, ticks, pre, EXACT, 6)).all()
    assert (base <= _counts(ids, ticks, suf, EXACT, 6)).all()
    rbase = _counts(ids, ticks, eps, RELAXED, 6)
    assert (rbase <= _counts(ids, ticks, pre, RELAXED, 6)).all()


# ---------------------------------------------------------------- P8 metamorphic
def test_gap_additivity_time_shift_projection():
    rng = np.random.default_rng(23)
    a_i, a_t = synth.sort_events(*synth.background(rng, np.full(5, 50.0), 50_000))
    b_i, b_t = synth.sort_events(*synth.background(rng, np.full(5, 50.0), 50_000))
    eps = _random_eps(rng, 120, 5, 5)
    shift = 50_000 + 2000
    ids = np.concatenate([a_i, b_i])
    ticks = np.concatenate([a_t, b_t + shift]).astype(np.int32)
    for mode in (EXACT, RELAXED):
        ca = _counts(a_i, a_t, eps, mode, 5)
        cb = _counts(b_i, b_t, eps, mode, 5)
        assert (_counts(ids, ticks, eps, mode, 5) == ca + cb).all()
        assert (_counts(a_i, a_t + 12345, eps, mode, 5) == ca).all()
        # projection: the same counts over the per-candidate sub-stream
        proj = oracle.count_episodes(ids, ticks, eps, mode=mode, num_types=5,
                                     projection=True, nthreads=2)
        assert (proj == ca + cb).all()
        # removing every event of a type outside the episode changes nothing
        for k, ep in enumerate(eps[:30]):
            keep = np.isin(ids, ep[0])
            assert _counts(ids[keep], ticks[keep], [ep], mode, 5)[0] == ca[k] + cb[k]


def test_projection_and_threads_match_plain_on_plain_config():
    s = synth.config_plain()
    c = s["candidates"]
    a = oracle.count(s["ids"], s["ticks"], 64, c["types"], c["len"], c["lo"], c["hi"],
                     EXACT, projection=False, nthreads=1)
    b = oracle.count(s["ids"], s["ticks"], 64, c["types"], c["len"], c["lo"], c["hi"],
                     EXACT, projection=True, nthreads=4)
    assert (a == b).all()


def test_two_pass_pipeline():
    s = synth.config_plain()
    c = s["candidates"]
    up, ex = oracle.two_pass(s["ids"], s["ticks"], 64, c["types"], c["len"], c["lo"], c["hi"],
                             s["theta"], projection=True)
    rx = oracle.count(s["ids"], s["ticks"], 64, c["types"], c["len"], c["lo"], c["hi"], RELAXED,
                      projection=True)
    full = oracle.count(s["ids"], s["ticks"], 64, c["types"], c["len"], c["lo"], c["hi"], EXACT,
                        projection=True)
    assert (up == rx).all()
    surv = up >= s["theta"]
    assert (ex[surv] == full[surv]).all() and (ex[~surv] == -1).all()
    # nothing frequent is lost by the elimination (Theorem of Sec. 5.3.2)
    assert ((full >= s["theta"]) <= surv).all()
    # the planted pairs are frequent
    for casc in s["cascades"]:
        for ep in synth.sub_episodes(casc, 2):
            m = ep[0][0] * 64 + ep[0][1]
            assert ex[m] >= 100
