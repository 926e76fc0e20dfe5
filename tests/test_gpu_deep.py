"""GPU parity for hops whose exact lists hold more than 8 live windows.

Algorithm 1 (Sec. 5.1) and Problem 1 (Sec. 2) accept any delay interval
0 <= lo < hi.  A list of hop (lo, hi] is a union of windows of which at most
hi/(hi-lo+1)+1 are live; narrow intervals far from 0 -- (190,200],
(199,200], (150,160] ticks -- exceed the 8 windows kept in registers and are
counted by the deep-class kernel (rings in device memory).  Every count here
is compared with the oracle, with such hops mixed with ordinary ones in one
call, through every entry point that counts exactly."""
import numpy as np
import pytest

import oracle
from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu, oracle_counts

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

EXACT, RELAXED = 0, 1
DEEP_IV = [(190, 200), (199, 200), (150, 160)]   # window bounds 19, 101, 15
PLAIN_IV = [(0, 50), (50, 100), (20, 30)]         # bounds 1, 2, 3
MIXED_IV = DEEP_IV + PLAIN_IV


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _stream(rng, n, T, mean_gap):
    ids = rng.integers(0, T, size=n).astype(np.int32)
    ticks = np.cumsum(rng.integers(0, 2 * mean_gap + 1, size=n)).astype(np.int32)
    return ids, ticks


def _mixed_cands(rng, T, M, nmax=5):
    eps = synth.random_episodes(rng, M, T, nmax, MIXED_IV, n_min=2)
    # shared-prefix runs with a deep hop in the prefix and in the last hop
    for iv in ((190, 200), (199, 200)):
        for last in range(T):
            for iv2 in MIXED_IV:
                eps.append(((1, 2, last), (iv[0], iv2[0]), (iv[1], iv2[1])))
    return synth.pack(eps)


def _count(ctx, ids, ticks, T, cand, mode, P):
    ctx.set_param(0, P)
    try:
        return ctx.count(ids, ticks, T, cand, mode).cpu().numpy()
    finally:
        ctx.set_param(0, 0)


@pytest.mark.parametrize("P", [0, 1, 2, 37])
def test_deep_hops_mixed_count(ctx, P):
    rng = np.random.default_rng(100 + P)
    T = 6
    ids_h, ticks_h = _stream(rng, 30000, T, 4)
    cand = _mixed_cands(rng, T, 1500)
    banner("deep hops mixed, M=%d, n=%d, P=%d" % (cand["M"], ids_h.size, P))
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    for mode in (EXACT, RELAXED):
        want = oracle_counts(ids_h, ticks_h, T, cand, mode)
        got = _count(ctx, ids, ticks, T, cand, mode, P)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (mode, bad[:5], got[bad[:5]], want[bad[:5]])
    assert want.max() > 0


def test_deep_rings_near_capacity(ctx):
    """A type firing every 3 ticks gives list (199,200] about 67 live
    single-tick windows (bound 201): the rings run near their capacity."""
    rng = np.random.default_rng(7)
    a_t = np.arange(0, 60000, 3)
    b_t = np.sort(rng.integers(0, 60000, 4000))
    ids_h, ticks_h = synth.sort_events(np.concatenate([np.zeros(a_t.size, np.int64),
                                                       np.ones(b_t.size, np.int64)]),
                                       np.concatenate([a_t, b_t]))
    eps = [((0, 1), (lo,), (hi,)) for lo, hi in DEEP_IV + [(180, 200), (100, 130), (299, 300)]]
    eps += [((0, 0), (lo,), (hi,)) for lo, hi in DEEP_IV]
    eps += [((0, 1, 0), (199, 10), (200, 40)), ((1, 0, 1), (150, 199), (160, 200))]
    cand = synth.pack(eps)
    banner("deep rings near capacity, n=%d" % ids_h.size)
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    want = oracle_counts(ids_h, ticks_h, 2, cand, EXACT)
    for P in (0, 5):
        got = _count(ctx, ids, ticks, 2, cand, EXACT, P)
        assert (got == want).all(), (P, got, want)
    assert (want > 0).sum() >= 5


def test_deep_rings_bounded_by_stream_and_chunked(ctx):
    """Intervals so narrow and far that the window bound (about 2^20) exceeds
    the stream length: each ring holds min(bound, n) windows, and the
    launches are cut into chunks of lanes (episodes of 8 nodes put 7 rings
    per lane), so some chunks end inside a tile."""
    rng = np.random.default_rng(11)
    T = 3
    ids_h, ticks_h = _stream(rng, 20000, T, 30)
    far = (1 << 20) - 1, 1 << 20
    eps = []
    for k in range(300):
        N = 2 + k % 7
        ty = tuple(int(x) for x in rng.integers(0, T, N))
        ivs = [far if rng.random() < 0.5 else (0, 60) for _ in range(N - 1)]
        eps.append((ty, tuple(a for a, _ in ivs), tuple(b for _, b in ivs)))
    # ordinary episodes that do count, in the same call
    eps += synth.random_episodes(rng, 200, T, 4, PLAIN_IV, n_min=2)
    cand = synth.pack(eps)
    banner("deep rings bounded by n, M=%d" % cand["M"])
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    want = oracle_counts(ids_h, ticks_h, T, cand, EXACT)
    got = _count(ctx, ids, ticks, T, cand, EXACT, 0)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])


def test_deep_two_pass_and_resume(ctx, fe):
    rng = np.random.default_rng(21)
    T = 5
    ids_h, ticks_h = _stream(rng, 20000, T, 4)
    cand = _mixed_cands(rng, T, 800)
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    banner("deep two-pass, M=%d" % cand["M"])
    for theta in (1, 40, 400):
        up, ex, ns = ctx.count_two_pass(ids, ticks, T, cand, theta)
        wu, we = oracle.two_pass(ids_h, ticks_h, T, cand["types"], cand["len"], cand["lo"],
                                 cand["hi"], theta, projection=True)
        assert (up.cpu().numpy() == wu).all(), theta
        assert (ex.cpu().numpy() == we).all(), theta
        assert int(ns.item()) == int((wu >= theta).sum())
    banner("deep resume")
    t = ctx.torch
    cd = ctx.cand_tensors(cand)
    cnt = t.zeros(cand["M"], dtype=t.int32, device=ctx.device)
    last = t.full((cand["M"],), -1, dtype=t.int32, device=ctx.device)
    prev = 0
    for cut in (0, 1, 64, 3000, 3001, 12000, ids_h.size):
        ctx.count_resume(ids[:cut], ticks[:cut], T, cd, EXACT, prev, cnt, last)
        want = oracle_counts(ids_h[:cut], ticks_h[:cut], T, cand, EXACT)
        got = cnt.cpu().numpy()
        assert (got == want).all(), (cut, np.nonzero(got != want)[0][:5])
        prev = cut


def test_deep_batched_and_served(ctx, fe):
    rng = np.random.default_rng(31)
    recs = []
    for r in range(3):
        T = 4 + r
        ids_h, ticks_h = _stream(rng, 8000 + 5000 * r, T, 4)
        recs.append({"ids": ids_h, "ticks": ticks_h, "num_types": T,
                     "candidates": _mixed_cands(rng, T, 300 + 100 * r), "theta": 5 + 10 * r})
    dev = []
    for rec in recs:
        ids, ticks = ctx.stream_tensors(rec["ids"], rec["ticks"])
        dev.append({"ids": ids, "ticks": ticks, "num_types": rec["num_types"],
                    "cand": ctx.cand_tensors(rec["candidates"]), "theta": rec["theta"]})
    banner("deep batched, %d recordings" % len(recs))
    b = fe.Batch(ctx, dev)
    for seg in (512, 32768):
        b.set_tuning(seg, 8)
        b.run()
        ctx.sync()
        for r, rec in enumerate(recs):
            c = rec["candidates"]
            wu, we = oracle.two_pass(rec["ids"], rec["ticks"], rec["num_types"], c["types"],
                                     c["len"], c["lo"], c["hi"], rec["theta"], projection=True)
            assert (b.upper[r].cpu().numpy() == wu).all(), (seg, r)
            assert (b.exact[r].cpu().numpy() == we).all(), (seg, r)
    b.close()

    banner("deep served")
    T = 6
    arrays = []
    for a in range(2):
        ids_h, ticks_h = _stream(rng, 20000, T, 4)
        arrays.append((ids_h, ticks_h))
    cand = _mixed_cands(rng, T, 500)
    sv = fe.Server(ctx, cand, [T, T], capacity=20016, hbm_budget=1 << 30, max_inflight=2,
                   max_round=4)
    for a, (ids_h, ticks_h) in enumerate(arrays):
        sv.append(a, ids_h, ticks_h)
    reqs = []
    for k in range(10):
        a = k % 2
        tk = arrays[a][1]
        t0 = int(rng.integers(0, int(tk[-1]) // 2))
        t1 = t0 + int(rng.integers(100, int(tk[-1]) // 2))
        reqs.append((a, t0, t1, 3 + k, sv.submit(a, t0, t1, 3 + k)))
    for a, t0, t1, theta, tkt in reqs:
        res = sv.wait(tkt)
        ids_h, ticks_h = arrays[a]
        lo_i, hi_i = np.searchsorted(ticks_h, t0, "left"), np.searchsorted(ticks_h, t1, "left")
        wu, we = oracle.two_pass(ids_h[lo_i:hi_i], ticks_h[lo_i:hi_i], T, cand["types"],
                                 cand["len"], cand["lo"], cand["hi"], theta, projection=True)
        assert res["status"] == fe.FE_OK
        assert (res["upper"] == wu).all() and (res["exact"] == we).all(), (a, t0, t1)
    sv.close()


def test_deep_interval_in_mining(ctx):
    from oracle import mine
    rng = np.random.default_rng(41)
    T = 5
    ids_h, ticks_h = _stream(rng, 12000, T, 3)
    intervals = [(0, 50), (190, 200)]
    theta = 60
    banner("mining with a deep interval")
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    got = ctx.mine(ids, ticks, T, intervals, theta, 4)
    want = mine.mine(ids_h, ticks_h, T, intervals, theta, 4)
    assert [lv["level"] for lv in got] == sorted(want)
    for lv in got:
        L = lv["level"]
        w = want[L]
        assert lv["n_candidates"] == len(w["candidates"]), L
        g = {(tuple(t), tuple(a), tuple(b)): (int(u), int(x))
             for t, a, b, u, x in zip(lv["types"], lv["lo"], lv["hi"], lv["upper"], lv["exact"])}
        wf = {ep: (int(w["upper"][k]), int(w["exact"][k]))
              for k, ep in enumerate(w["candidates"]) if ep in w["frequent"]}
        assert g == wf, L
    deep_freq = sum(1 for lv in got for b in lv["hi"] if 200 in b.tolist())
    assert deep_freq > 0
