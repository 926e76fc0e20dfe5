"""GPU parity: every count from the HIP library equals the CPU oracle's,
bit for bit, on seeded synthetic inputs (fe_count, fe_count_two_pass,
fe_mine through the C ABI)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu, oracle_counts

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

EXACT, RELAXED = 0, 1


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _dev(ctx, s):
    return ctx.stream_tensors(s["ids"], s["ticks"])


def _count(ctx, ids, ticks, num_types, cand, mode, P=0):
    ctx.set_param(0, P)
    try:
        return ctx.count(ids, ticks, num_types, cand, mode).cpu().numpy()
    finally:
        ctx.set_param(0, 0)


# ---------------------------------------------------------------- plain config
@pytest.fixture(scope="module")
def plain():
    return synth.config_plain()


@pytest.mark.parametrize("mode", [RELAXED, EXACT])
def test_plain_all_pairs(ctx, plain, mode):
    banner("plain config, 4096 pairs, mode=%d" % mode)
    ids, ticks = _dev(ctx, plain)
    got = _count(ctx, ids, ticks, 64, plain["candidates"], mode)
    want = oracle_counts(plain["ids"], plain["ticks"], 64, plain["candidates"], mode)
    assert (got == want).all(), np.nonzero(got != want)[0][:10]


@pytest.mark.parametrize("P", [1, 2, 3, 64, 1024])
def test_plain_segment_sweep(ctx, plain, P):
    banner("plain config, P=%d" % P)
    ids, ticks = _dev(ctx, plain)
    for mode in (RELAXED, EXACT):
        got = _count(ctx, ids, ticks, 64, plain["candidates"], mode, P)
        want = oracle_counts(plain["ids"], plain["ticks"], 64, plain["candidates"], mode)
        assert (got == want).all(), (mode, np.nonzero(got != want)[0][:10])


def test_plain_two_pass(ctx, plain):
    banner("plain config two-pass")
    ids, ticks = _dev(ctx, plain)
    c = plain["candidates"]
    up, ex, ns = ctx.count_two_pass(ids, ticks, 64, c, plain["theta"])
    wu, we = oracle.two_pass(plain["ids"], plain["ticks"], 64, c["types"], c["len"], c["lo"],
                             c["hi"], plain["theta"], projection=True)
    assert (up.cpu().numpy() == wu).all()
    assert (ex.cpu().numpy() == we).all()
    assert int(ns.item()) == int((wu >= plain["theta"]).sum())


# ---------------------------------------------------------------- tiny fuzz
TINY_IV = [(0, 1), (0, 3), (1, 3), (2, 5), (3, 4)]   # depth bounds 1, 1, 2, 2, 3


def _tiny_cands(n_types):
    eps = [((e,), (), ()) for e in range(n_types)]
    for N in (2, 3):
        for ty in itertools.product(range(n_types), repeat=N):
            for ivs in itertools.product(TINY_IV, repeat=N - 1):
                if N == 3 and (ivs[0] == ivs[1]) is False and ty[0] > 1:
                    continue
                eps.append((ty, tuple(l for l, _ in ivs), tuple(h for _, h in ivs)))
    return synth.pack(eps)


def test_tiny_fuzz_streams(ctx):
    rng = np.random.default_rng(1234)
    cand = _tiny_cands(3)
    banner("tiny fuzz, %d candidates" % cand["M"])
    for trial in range(60):
        n = int(rng.integers(0, 80))
        ids_h, ticks_h = synth.tiny_stream(rng, n, 3, 3)
        ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
        for mode in (RELAXED, EXACT):
            want = oracle_counts(ids_h, ticks_h, 3, cand, mode, projection=False)
            for P in (1, 2, 5, max(n, 1)):
                got = _count(ctx, ids, ticks, 3, cand, mode, P)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (trial, n, mode, P, bad[:5])


# ---------------------------------------------------------------- sizes, depths
DEPTH_IV = [(0, 50), (50, 100), (100, 150), (170, 200), (20, 30)]


def test_mixed_sizes_and_depth_classes(ctx):
    rng = np.random.default_rng(77)
    ids_h, ticks_h = synth.sort_events(*synth.background(rng, np.full(10, 60.0), 300_000))
    eps = synth.random_episodes(rng, 3000, 10, 8, DEPTH_IV, n_min=1)
    cand = synth.pack(eps)
    banner("mixed N 1..8, depth classes, n=%d" % ids_h.size)
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    for mode in (RELAXED, EXACT):
        want = oracle_counts(ids_h, ticks_h, 10, cand, mode)
        for P in (0, 1, 37):
            got = _count(ctx, ids, ticks, 10, cand, mode, P)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (mode, P, bad[:5], got[bad[:5]], want[bad[:5]])


def test_slot_overflow_falls_back_exactly(ctx):
    """Bursts of many same-tick events of the last type put more than the
    kept number of restart slots into a look-back."""
    rng = np.random.default_rng(5)
    bi, bt = synth.background(rng, np.full(4, 30.0), 200_000)
    burst_t = np.repeat(np.sort(rng.integers(0, 200_000, 400)), 6)
    ids_h, ticks_h = synth.sort_events(np.concatenate([bi, np.full(burst_t.size, 3)]),
                                       np.concatenate([bt, burst_t]))
    eps = [((a, 3), (0,), (h,)) for a in range(4) for h in (5, 50, 300)]
    eps += [((a, b, 3), (0, 10), (100, 200)) for a in range(4) for b in range(4)]
    cand = synth.pack(eps)
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    banner("slot overflow bursts")
    for mode in (RELAXED, EXACT):
        want = oracle_counts(ids_h, ticks_h, 4, cand, mode)
        for P in (50, 400, 3000):
            got = _count(ctx, ids, ticks, 4, cand, mode, P)
            assert (got == want).all(), (mode, P)


# ---------------------------------------------------------------- boundary
def test_error_codes_and_degenerate_inputs(ctx, fe):
    banner("error codes")
    ids, ticks = ctx.stream_tensors([0, 1, 0, 1], [0, 5, 3, 9])
    cand = synth.pack([((0, 1), (0,), (10,))])
    with pytest.raises(fe.FeError) as e:
        ctx.count(ids, ticks, 2, cand, EXACT)
    assert e.value.code == fe.FE_EUNSORTED
    ids, ticks = ctx.stream_tensors([0, 7, 0], [0, 5, 9])
    with pytest.raises(fe.FeError) as e:
        ctx.count(ids, ticks, 2, cand, EXACT)
    assert e.value.code == fe.FE_ERANGE
    ids, ticks = ctx.stream_tensors([0, 1, 0], [0, 5, 9])
    for bad in ([((0, 1), (5,), (5,))], [((0, 1), (-1,), (5,))], [((0, 4), (0,), (5,))],
                [((0, 1), (0,), (1 << 30,))]):
        with pytest.raises(fe.FeError) as e:
            ctx.count(ids, ticks, 2, synth.pack(bad), EXACT)
        assert e.value.code == fe.FE_EINVAL
    # narrow intervals far from 0 are valid hops (Problem 1): counted exactly
    ids2, ticks2 = ctx.stream_tensors([0, 1, 0, 1, 1], [0, 195, 300, 499, 500])
    narrow = synth.pack([((0, 1), (190,), (200,)), ((0, 1), (199,), (200,)),
                         ((0, 1), (194,), (195,)), ((0, 1), (150,), (160,))])
    for mode, want in ((EXACT, [2, 1, 1, 0]), (RELAXED, [2, 2, 1, 0])):
        got = ctx.count(ids2, ticks2, 2, narrow, mode).cpu().numpy()
        assert got.tolist() == want, (mode, got)
        assert got.tolist() == oracle_counts(np.array([0, 1, 0, 1, 1]),
                                             np.array([0, 195, 300, 499, 500]), 2, narrow,
                                             mode).tolist()
    # the context still works after errors
    assert ctx.count(ids, ticks, 2, cand, EXACT)[0].item() == 1
    # empty stream: all zeros
    e_ids, e_ticks = ctx.stream_tensors(np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert (ctx.count(e_ids, e_ticks, 2, cand, EXACT).cpu().numpy() == 0).all()
    up, ex, ns = ctx.count_two_pass(e_ids, e_ticks, 2, cand, 0)
    assert up.item() == 0 and ex.item() == 0 and ns.item() == 1
    up, ex, ns = ctx.count_two_pass(e_ids, e_ticks, 2, cand, 1)
    assert up.item() == 0 and ex.item() == -1 and ns.item() == 0


# ---------------------------------------------------------------- mining
def test_mining_matches_oracle_small(ctx):
    from oracle import mine
    s = synth.config_mining(n_neurons=16, rate_hz=20.0, duration_s=90.0, n_cascades=3, tag=52)
    banner("mining small: n=%d theta=%d" % (s["ids"].size, s["theta"]))
    ids, ticks = _dev(ctx, s)
    got = ctx.mine(ids, ticks, s["num_types"], s["intervals"], s["theta"], 6)
    want = mine.mine(s["ids"], s["ticks"], s["num_types"], s["intervals"], s["theta"], 6)
    # the same levels (both stop after the first level without a frequent
    # episode, or at the first level without candidates)
    assert [lv["level"] for lv in got] == sorted(want)
    for lv in got:
        L = lv["level"]
        w = want[L]
        assert lv["n_candidates"] == len(w["candidates"]), L
        if L > 1 and lv["passes"] == 2:
            assert lv["n_survivors"] == int((w["upper"] >= s["theta"]).sum()), L
        elif L > 1:
            assert lv["n_survivors"] == lv["n_candidates"], L
        g = {(tuple(t), tuple(a), tuple(b)): (int(u), int(x))
             for t, a, b, u, x in zip(lv["types"], lv["lo"], lv["hi"], lv["upper"], lv["exact"])}
        wf = {}
        for k, ep in enumerate(w["candidates"]):
            if ep in w["frequent"]:
                wf[ep] = (int(w["upper"][k]), int(w["exact"][k]))
        assert g == wf, (L, len(g), len(wf))
