"""GPU parity of the exact Map for waves of join siblings (candidates that
share every node type but the last and every hop but the last), where lists
0..N-3 are kept once per wave (FE_PARAM_SHARED_LISTS): whole-stream exact
counts (P = 1) equal the CPU oracle's bit for bit and the per-candidate
lists' counts, for N = 3..8; with repeated types in the shared prefix and
last types equal to a shared type; with ties in the ticks; with type ids
above 63 (hash collisions in the last node's table); with bursts that
overflow the 64-entry rings (the tile is then counted the general way); on
tiny, ragged and empty streams; and for runs of siblings over several tiles
(whole tiles, a padded remainder tile, remainders packed with other runs'
into mixed tiles)."""
import numpy as np
import pytest

from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu, oracle_counts

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

EXACT = 0
# hops whose window bound hi/(hi-lo+1)+1 is at most 2: one list-depth class
PRE_HOPS = [(50, 100), (100, 200), (10, 40)]
LAST_HOPS = [(50, 100), (100, 200), (10, 40), (0, 30), (0, 1)]


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _count(ctx, fe, ids, ticks, num_types, cand, shared):
    ctx.set_param(fe.PARAM_SEGMENTS, 1)
    ctx.set_param(fe.PARAM_SHARED_LISTS, shared)
    try:
        return ctx.count(ids, ticks, num_types, cand, EXACT).cpu().numpy()
    finally:
        ctx.set_param(fe.PARAM_SEGMENTS, 0)
        ctx.set_param(fe.PARAM_SHARED_LISTS, 1)


def _siblings(rng, N, runs, num_types, repeat=False, last_pool=None, sizes=None):
    """runs x 64 candidates (or runs of the given sizes); each run shares N-1
    node types and N-2 hops, each lane draws its last type and last hop."""
    eps = []
    for r in range(runs if sizes is None else len(sizes)):
        pre = [int(x) for x in rng.integers(0, num_types, N - 1)]
        if repeat and N >= 3:  # a type repeated inside the shared prefix
            pre[1] = pre[0]
        hops = [PRE_HOPS[int(rng.integers(len(PRE_HOPS)))] for _ in range(N - 2)]
        for _ in range(64 if sizes is None else sizes[r]):
            if last_pool is None:
                last = int(rng.integers(num_types))
            else:
                last = int(rng.choice(last_pool(pre)))
            lh = LAST_HOPS[int(rng.integers(len(LAST_HOPS)))]
            iv = hops + [lh]
            eps.append((tuple(pre) + (last,), tuple(a for a, _ in iv), tuple(b for _, b in iv)))
    return synth.pack(eps)


def _stream(rng, n, num_types, mean_gap=6, weights=None):
    ids = rng.choice(num_types, size=n, p=weights).astype(np.int32)
    ticks = np.cumsum(rng.integers(0, 2 * mean_gap + 1, size=n)).astype(np.int32)
    return ids, ticks


def _check(ctx, fe, ids_h, ticks_h, num_types, cand, what, nonvacuous=True):
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    want = oracle_counts(ids_h, ticks_h, num_types, cand, EXACT)
    for shared in (1, 0):
        got = _count(ctx, fe, ids, ticks, num_types, cand, shared)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (what, shared, bad[:5], got[bad[:5]], want[bad[:5]])
    if nonvacuous:
        assert (want > 0).sum() >= cand["M"] // 20, what  # the case is not vacuous


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7, 8])
def test_join_siblings(ctx, fe, N):
    rng = np.random.default_rng(500 + N)
    nt = 6 if N <= 4 else 4
    ids_h, ticks_h = _stream(rng, 30_000, nt, mean_gap=8 if N <= 5 else 3)
    cand = _siblings(rng, N, 8, nt)
    banner("join siblings: N=%d, %d candidates, n=%d" % (N, cand["M"], ids_h.size))
    _check(ctx, fe, ids_h, ticks_h, nt, cand, "N=%d" % N)


@pytest.mark.parametrize("N", [3, 4, 5])
def test_repeated_and_last_in_prefix(ctx, fe, N):
    rng = np.random.default_rng(600 + N)
    ids_h, ticks_h = _stream(rng, 25_000, 5)
    cand = _siblings(rng, N, 8, 5, repeat=True, last_pool=lambda pre: pre)
    banner("repeated prefix types, last type in the prefix: N=%d" % N)
    _check(ctx, fe, ids_h, ticks_h, 5, cand, "repeat N=%d" % N)


def test_ties_in_ticks(ctx, fe):
    rng = np.random.default_rng(71)
    n = 30_000
    ids_h = rng.integers(0, 5, n).astype(np.int32)
    ticks_h = np.cumsum(rng.integers(0, 3, n) * 10).astype(np.int32)  # many equal ticks
    cand = _siblings(rng, 4, 8, 5)
    banner("ties in ticks")
    _check(ctx, fe, ids_h, ticks_h, 5, cand, "ties")


def test_type_ids_above_63(ctx, fe):
    rng = np.random.default_rng(72)
    nt = 200
    hot = np.array([3, 67, 131, 195, 10, 74, 138, 199])  # 3, 67, 131, 195 share a hash
    w = np.full(nt, 0.2 / (nt - hot.size))
    w[hot] = 0.1
    w /= w.sum()
    ids_h, ticks_h = _stream(rng, 40_000, nt, mean_gap=2, weights=w)
    cand = _siblings(rng, 4, 6, nt, last_pool=lambda pre: hot)
    # shared prefixes from the hot ids too
    t = cand["types"]
    for r in range(t.shape[0] // 64):
        t[r * 64:(r + 1) * 64, :3] = rng.choice(hot, 3)
    banner("type ids above 63")
    _check(ctx, fe, ids_h, ticks_h, nt, cand, "hash")


def test_ring_overflow_falls_back(ctx, fe):
    # node 0's type fires 200 times within a few ticks, again and again:
    # more list-0 entries than a ring holds can still pass the next hop
    rng = np.random.default_rng(73)
    parts_i, parts_t, t0 = [], [], 0
    for _ in range(40):
        k = int(rng.integers(150, 260))
        parts_i.append(np.zeros(k, np.int32))
        parts_t.append(t0 + np.sort(rng.integers(0, 20, k)).astype(np.int32))
        t0 += 20
        m = int(rng.integers(100, 300))
        parts_i.append(rng.integers(1, 4, m).astype(np.int32))
        parts_t.append(t0 + np.cumsum(rng.integers(0, 4, m)).astype(np.int32))
        t0 = int(parts_t[-1][-1]) + 1
    ids_h, ticks_h = np.concatenate(parts_i), np.concatenate(parts_t)
    eps = []
    for r in range(4):
        for j in range(64):
            eps.append(((0, 1 + r % 3, 1 + j % 3), (10, int(j % 6)), (60, int(j % 6) + 40)))
    cand = synth.pack(eps)
    banner("ring overflow: n=%d" % ids_h.size)
    _check(ctx, fe, ids_h, ticks_h, 4, cand, "overflow")


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000])
def test_tiny_and_ragged(ctx, fe, n):
    rng = np.random.default_rng(80 + n)
    ids_h, ticks_h = _stream(rng, n, 3, mean_gap=20)
    cand = _siblings(rng, 3, 2, 3)
    _check(ctx, fe, ids_h, ticks_h, 3, cand, "n=%d" % n, nonvacuous=n >= 1000)


# runs over 2, 3 and 17 tiles (a remainder of at least 32 gets a padded tile
# of its own, a shorter one is packed with others), one of 64 and short ones
RUN_SIZES = [100, 64, 130, 65 + 32, 200, 20, 64 * 17 + 40, 128, 7, 64 * 3]


@pytest.mark.parametrize("N", [3, 4, 6])
def test_sibling_runs_over_several_tiles(ctx, fe, N):
    rng = np.random.default_rng(900 + N)
    nt = 6 if N <= 4 else 4
    ids_h, ticks_h = _stream(rng, 20_000, nt, mean_gap=8 if N <= 4 else 3)
    cand = _siblings(rng, N, 0, nt, sizes=RUN_SIZES)
    banner("sibling runs over several tiles: N=%d, %d candidates" % (N, cand["M"]))
    _check(ctx, fe, ids_h, ticks_h, nt, cand, "runs N=%d" % N)


@pytest.mark.parametrize("seed", range(12))
def test_random_sibling_runs(ctx, fe, seed):
    """Random N (3..6), hops (some with lo > 0 and narrow windows), run
    sizes, stream lengths (not multiples of 64) and burstiness; shared
    lists on and off against the oracle."""
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.integers(3, 7))
    nt = int(rng.integers(3, 9))
    n = int(rng.integers(2_000, 12_000))
    gaps = rng.integers(0, int(rng.integers(2, 16)), n)
    if seed % 3 == 0:  # bursts: runs of equal ticks
        gaps[rng.random(n) < 0.5] = 0
    ids_h = rng.integers(0, nt, n).astype(np.int32)
    ticks_h = np.cumsum(gaps).astype(np.int32)
    hop_pool = [(0, 5), (0, 30), (10, 40), (50, 100), (5, 8), (20, 25)]
    eps = []
    for _ in range(int(rng.integers(2, 6))):
        pre = [int(x) for x in rng.integers(0, nt, N - 1)]
        hops = [hop_pool[int(rng.integers(len(hop_pool)))] for _ in range(N - 2)]
        for _ in range(int(rng.integers(20, 150))):
            lh = hop_pool[int(rng.integers(len(hop_pool)))]
            iv = hops + [lh]
            eps.append((tuple(pre) + (int(rng.integers(nt)),), tuple(a for a, _ in iv),
                        tuple(b for _, b in iv)))
    cand = synth.pack(eps)
    banner("random sibling runs: seed=%d N=%d n=%d M=%d" % (seed, N, n, cand["M"]))
    _check(ctx, fe, ids_h, ticks_h, nt, cand, "seed=%d" % seed, nonvacuous=False)
