"""GPU parity of the per-type dispatch Map path (FE_PARAM_TYPE_DISPATCH):
with it on and off, whole-stream counts (P = 1) equal the CPU oracle's bit for
bit, for waves whose candidates share their first N-1 types (runs of 64 in
input order) and for waves that do not; with type ids that collide in the
64-entry type hash; with last types equal to a shared type; with blocks
crowded with shared-type events; and on ragged and tiny streams."""
import numpy as np
import pytest

from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu, oracle_counts

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

EXACT, RELAXED = 0, 1
# list depths 2, 2 and 3 (exact machines with 2 and 4 windows)
IV_D2 = [(50, 100), (100, 200), (60, 110)]


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _count(ctx, fe, ids, ticks, num_types, cand, mode, dispatch):
    ctx.set_param(fe.PARAM_SEGMENTS, 1)
    ctx.set_param(fe.PARAM_TYPE_DISPATCH, dispatch)
    try:
        return ctx.count(ids, ticks, num_types, cand, mode).cpu().numpy()
    finally:
        ctx.set_param(fe.PARAM_SEGMENTS, 0)
        ctx.set_param(fe.PARAM_TYPE_DISPATCH, 1)


def _prefix_runs(rng, N, runs, prefixes, last_pool, ivs=IV_D2):
    """runs x 64 candidates; run r shares the node types prefixes[r % len]
    (N-1 of them); each lane draws its last type and intervals."""
    eps = []
    for r in range(runs):
        pre = prefixes[r % len(prefixes)]
        for _ in range(64):
            last = int(rng.choice(last_pool))
            iv = [ivs[int(rng.integers(len(ivs)))] for _ in range(N - 1)]
            eps.append((tuple(pre) + (last,), tuple(a for a, _ in iv), tuple(b for _, b in iv)))
    return synth.pack(eps)


def _stream(rng, n, num_types, weights=None, mean_gap=8):
    ids = rng.choice(num_types, size=n, p=weights).astype(np.int32)
    ticks = np.cumsum(rng.integers(0, 2 * mean_gap + 1, size=n)).astype(np.int32)
    return ids, ticks


def _check(ctx, fe, ids_h, ticks_h, num_types, cand, what):
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    for mode in (RELAXED, EXACT):
        want = oracle_counts(ids_h, ticks_h, num_types, cand, mode)
        for dispatch in (1, 0):
            got = _count(ctx, fe, ids, ticks, num_types, cand, mode, dispatch)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (what, mode, dispatch, bad[:5], got[bad[:5]], want[bad[:5]])
        assert (want > 0).any(), what  # the case is not vacuous


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_shared_prefix_runs(ctx, fe, N):
    rng = np.random.default_rng(100 + N)
    ids_h, ticks_h = _stream(rng, 40_000, 16)
    prefixes = [tuple(int(x) for x in rng.integers(0, 16, N - 1)) for _ in range(6)]
    cand = _prefix_runs(rng, N, 12, prefixes, np.arange(16))
    banner("shared-prefix runs: N=%d, %d candidates, n=%d" % (N, cand["M"], ids_h.size))
    _check(ctx, fe, ids_h, ticks_h, 16, cand, "N=%d" % N)


def test_type_hash_collisions(ctx, fe):
    # types t, t+64, t+128 share a hash; prefixes and last types mix them,
    # and some last types equal a shared type
    rng = np.random.default_rng(7)
    T = 200
    w = np.full(T, 1.0)
    for t in (5, 69, 133, 197, 9, 73):
        w[t] = 40.0
    ids_h, ticks_h = _stream(rng, 60_000, T, w / w.sum())
    prefixes = [(5, 69, 133), (69, 5, 9), (133, 197, 73), (9, 9, 5)]
    pool = np.array([5, 69, 133, 197, 9, 73, 137, 1, 65, 129])
    cand = _prefix_runs(rng, 4, 8, prefixes, pool)
    banner("hash collisions: %d candidates, n=%d" % (cand["M"], ids_h.size))
    _check(ctx, fe, ids_h, ticks_h, T, cand, "collisions")


def test_crowded_prefix_blocks(ctx, fe):
    # most events carry a shared type: blocks are stepped event by event
    rng = np.random.default_rng(11)
    w = np.full(32, 1.0)
    w[[3, 4, 5]] = 60.0
    ids_h, ticks_h = _stream(rng, 30_000, 32, w / w.sum(), mean_gap=30)
    cand = _prefix_runs(rng, 4, 6, [(3, 4, 5), (5, 3, 4)], np.arange(32))
    banner("crowded prefix blocks: %d candidates" % cand["M"])
    _check(ctx, fe, ids_h, ticks_h, 32, cand, "crowded")


@pytest.mark.parametrize("N,prefixes", [
    (3, [(2, 2), (2, 5), (5, 2)]),
    (4, [(1, 2, 2), (2, 2, 2), (2, 2, 1), (1, 2, 1)]),
    (5, [(1, 1, 2, 2), (2, 1, 2, 1)]),
])
def test_repeated_prefix_types(ctx, fe, N, prefixes):
    # node N-3 and node N-2 share a type, or node N-2's type recurs earlier:
    # an event can both close a span and be the block's first node N-3 event;
    # dense prefix types keep list N-3 alive across some block starts and
    # not others
    rng = np.random.default_rng(300 + N)
    w = np.full(24, 1.0)
    w[[1, 2, 5]] = 12.0
    ids_h, ticks_h = _stream(rng, 40_000, 24, w / w.sum(), mean_gap=12)
    cand = _prefix_runs(rng, N, 4 * len(prefixes), prefixes, np.arange(24),
                        ivs=[(0, 50), (50, 100), (100, 200), (20, 60)])
    banner("repeated prefix types: N=%d, %d candidates" % (N, cand["M"]))
    _check(ctx, fe, ids_h, ticks_h, 24, cand, "repeated N=%d" % N)


def test_mixed_waves_and_ragged_streams(ctx, fe):
    # random candidates (no shared prefix: lane-by-lane dispatch) next to
    # shared-prefix runs, over streams of every length class around a block
    rng = np.random.default_rng(23)
    eps = synth.random_episodes(rng, 700, 12, 4, IV_D2, n_min=1)
    runs = _prefix_runs(rng, 4, 3, [(1, 2, 3)], np.arange(12))
    eps += [(tuple(runs["types"][m, :4]), tuple(runs["lo"][m, :3]), tuple(runs["hi"][m, :3]))
            for m in range(runs["M"])]
    cand = synth.pack(eps)
    for n in (1, 2, 63, 64, 65, 127, 129, 1000, 4097, 20_001):
        ids_h, ticks_h = _stream(rng, n, 12, mean_gap=40)
        ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
        banner("mixed waves: n=%d, %d candidates" % (n, cand["M"]))
        for mode in (RELAXED, EXACT):
            want = oracle_counts(ids_h, ticks_h, 12, cand, mode)
            for dispatch in (1, 0):
                got = _count(ctx, fe, ids, ticks, 12, cand, mode, dispatch)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (n, mode, dispatch, bad[:5], got[bad[:5]], want[bad[:5]])


def test_mining_same_with_and_without_dispatch(ctx, fe):
    s = synth.config_mining(duration_s=60.0)
    banner("mining 60 s: n=%d theta=%d" % (s["ids"].size, s["theta"]))
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    res = {}
    for dispatch in (1, 0):
        ctx.set_param(fe.PARAM_TYPE_DISPATCH, dispatch)
        try:
            out = ctx.mine(ids, ticks, s["num_types"], s["intervals"], s["theta"], 5)
        finally:
            ctx.set_param(fe.PARAM_TYPE_DISPATCH, 1)
        res[dispatch] = out
    assert len(res[0]) == len(res[1])
    for a, b in zip(res[0], res[1]):
        for k in ("types", "lo", "hi", "upper", "exact"):
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (a["level"], k)


def test_hybrid_crossover_rule(ctx, fe):
    # below the crossover C(N) = A/N + B tiles the count is segmented (P >= 2),
    # at or above it whole-stream (P = 1); each counter has its own A and B;
    # the counts are the same
    rng = np.random.default_rng(41)
    ids_h, ticks_h = _stream(rng, 50_000, 16)
    # 40 tiles in one group (one list-depth class)
    cand = _prefix_runs(rng, 4, 40, [(1, 2, 3), (4, 5, 6)], np.arange(16),
                        ivs=[(50, 100), (100, 200)])
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    keys = (fe.PARAM_CROSSOVER_A, fe.PARAM_CROSSOVER_B, fe.PARAM_CROSSOVER_A_RELAXED,
            fe.PARAM_CROSSOVER_B_RELAXED)
    saved = {p: ctx.get_param(p) for p in keys}
    A0, B0, AR, BR = (saved[p] for p in keys)
    assert A0 / 4 + B0 > 40 and AR / 4 + BR > 40
    want = {m: oracle_counts(ids_h, ticks_h, 16, cand, m) for m in (EXACT, RELAXED)}

    def run(mode):
        got = ctx.count(ids, ticks, 16, cand, mode).cpu().numpy()
        assert (got == want[mode]).all()
        return ctx.stats()["segments_max"]
    try:
        assert run(EXACT) >= 2 and run(RELAXED) >= 2
        ctx.set_param(fe.PARAM_CROSSOVER_A, 0)
        ctx.set_param(fe.PARAM_CROSSOVER_B, 40)   # C(4) = 40 tiles: whole stream
        assert run(EXACT) == 1
        assert run(RELAXED) >= 2                  # the relaxed rule is its own
        ctx.set_param(fe.PARAM_CROSSOVER_B, 41)
        assert run(EXACT) >= 2
        ctx.set_param(fe.PARAM_CROSSOVER_A_RELAXED, -40)
        ctx.set_param(fe.PARAM_CROSSOVER_B_RELAXED, 50)   # C(4) = 40
        assert run(RELAXED) == 1
        ctx.set_param(fe.PARAM_CROSSOVER_B_RELAXED, 51)
        assert run(RELAXED) >= 2
        with pytest.raises(fe.FeError):
            ctx.set_param(fe.PARAM_CROSSOVER_B, -1)   # only A may be negative
    finally:
        for p, v in saved.items():
            ctx.set_param(p, v)


def test_one_pass_mining_same_result(ctx, fe):
    # Algorithm 1 over every candidate (no elimination), two passes at every
    # level, and the per-level decision from a sampled relaxed pass find the
    # same frequent episodes with the same exact counts
    s = synth.config_mining(duration_s=60.0)
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    saved = {p: ctx.get_param(p) for p in (fe.PARAM_ELIMINATION, fe.PARAM_SAMPLE_MIN,
                                            fe.PARAM_PASS1_COST)}
    res = {}
    try:
        ctx.set_param(fe.PARAM_SAMPLE_MIN, 1000)
        for key, elim, cost in (("two", 1, 800), ("one", 0, 800), ("rule_two", 2, 0),
                                ("rule_one", 2, 1000), ("rule", 2, 800)):
            ctx.set_param(fe.PARAM_ELIMINATION, elim)
            ctx.set_param(fe.PARAM_PASS1_COST, cost)
            res[key] = ctx.mine(ids, ticks, s["num_types"], s["intervals"], s["theta"], 5)
    finally:
        for p, v in saved.items():
            ctx.set_param(p, v)
    for key in res:
        assert [L["level"] for L in res[key]] == [L["level"] for L in res["two"]], key
        for a, b in zip(res["two"], res[key]):
            for k in ("types", "lo", "hi", "exact", "n_frequent", "n_candidates"):
                assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (key, a["level"], k)
            if a["level"] < 2:
                continue
            if b["passes"] == 1:
                assert (np.asarray(b["upper"]) == -1).all()
                assert b["n_survivors"] == b["n_candidates"]
            else:
                assert np.array_equal(a["upper"], b["upper"]) and \
                    a["n_survivors"] == b["n_survivors"], (key, a["level"])
    # the rule: two passes when the sampled survivor fraction is below
    # 1 - cost (no sample and one pass when cost >= 1); levels below the
    # sampling size take two passes
    for key, cost in (("rule_two", 0), ("rule_one", 1000), ("rule", 800)):
        big = [L for L in res[key] if L["level"] >= 2 and L["n_candidates"] >= 1000]
        assert big, key
        for L in res[key]:
            if L["level"] < 2:
                continue
            if L["n_candidates"] < 1000:
                want = 2
            elif cost >= 1000:
                assert L["sample_n"] == 0, (key, L["level"])
                want = 1
            else:
                assert L["sample_n"] > 0, (key, L["level"])
                want = 2 if L["sample_kept"] < (1 - cost / 1000) * L["sample_n"] else 1
            assert L["passes"] == want, (key, L["level"])
    assert any(L["passes"] == 2 for L in res["rule_two"] if L["sample_n"])
    assert all(L["passes"] == 1 for L in res["one"] if L["level"] >= 2)


def _mine_with(ctx, fe, s, intervals, theta, max_level, htile, elim):
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    h0 = ctx.get_param(fe.PARAM_HOST_TILING)
    e0 = ctx.get_param(fe.PARAM_ELIMINATION)
    ctx.set_param(fe.PARAM_HOST_TILING, htile)
    ctx.set_param(fe.PARAM_ELIMINATION, elim)
    try:
        return ctx.mine(ids, ticks, s["num_types"], intervals, theta, max_level)
    finally:
        ctx.set_param(fe.PARAM_HOST_TILING, h0)
        ctx.set_param(fe.PARAM_ELIMINATION, e0)


def _same_levels(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        for k in ("level", "n_candidates", "n_survivors", "n_frequent"):
            assert x[k] == y[k], (x["level"], k, x[k], y[k])
        for k in ("types", "lo", "hi", "upper", "exact"):
            assert np.array_equal(np.asarray(x[k]), np.asarray(y[k])), (x["level"], k)


@pytest.mark.parametrize("elim", [1, 0])
def test_device_tiling_same_as_host(ctx, fe, elim):
    # pruning and tiling on the device (default) against the host tiler:
    # the same survivors, frequent episodes and counts at every level
    s = synth.config_mining(duration_s=60.0)
    banner("device vs host tiling, mining 60 s, elimination=%d" % elim)
    dev = _mine_with(ctx, fe, s, s["intervals"], s["theta"], 5, 0, elim)
    host = _mine_with(ctx, fe, s, s["intervals"], s["theta"], 5, 1, elim)
    _same_levels(dev, host)
    assert any(L["n_frequent"] > 0 for L in dev if L["level"] >= 3)


def test_device_tiling_depth_classes(ctx, fe):
    # intervals of list-depth classes 0, 1 and 2 in one level, a low threshold
    # (most candidates frequent, so a lost or doubled lane would show), and
    # short sibling runs (16 types): full, padded and packed tiles per class
    s = synth.config_mining(n_neurons=16, duration_s=40.0)
    ivs = [(0, 50), (50, 100), (100, 150), (20, 30)]
    banner("device vs host tiling, depth classes, n=%d" % s["ids"].size)
    dev = _mine_with(ctx, fe, s, ivs, 10, 4, 0, 1)
    host = _mine_with(ctx, fe, s, ivs, 10, 4, 1, 1)
    _same_levels(dev, host)
    assert dev[-1]["level"] == 4 and dev[-1]["n_frequent"] > 1000
