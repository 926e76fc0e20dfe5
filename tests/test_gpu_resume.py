"""GPU parity of incremental counting (fe_count_resume): a stream counted in
consecutive partitions, carrying each candidate's count and last completion
index, gives after every partition exactly the oracle's count over the
stream so far; the carried index is the last completion's."""
import numpy as np
import pytest

import oracle
from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu, oracle_counts

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

EXACT, RELAXED = 0, 1
IVS = [(0, 40), (30, 80), (60, 140), (100, 130)]   # depth classes 1, 2, 3 and 4


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


def _cands(rng, T):
    eps = synth.random_episodes(rng, 600, T, 5, IVS, n_min=1)
    pre = (1, 2, 3)
    for _ in range(128):   # two shared-prefix tiles
        iv = [IVS[int(rng.integers(len(IVS)))] for _ in range(3)]
        eps.append((pre + (int(rng.integers(T)),), tuple(a for a, _ in iv),
                    tuple(b for _, b in iv)))
    return synth.pack(eps)


def _run(ctx, fe, ids_h, ticks_h, T, cand, mode, cuts, dispatch):
    t = ctx.torch
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    M = cand["M"]
    cnt = t.zeros(M, dtype=t.int32, device=ctx.device)
    last = t.full((M,), -1, dtype=t.int32, device=ctx.device)
    ctx.set_param(fe.PARAM_TYPE_DISPATCH, dispatch)
    try:
        prev = 0
        for cut in cuts:
            ctx.count_resume(ids[:cut], ticks[:cut], T, cand, mode, prev, cnt, last)
            want = oracle_counts(ids_h[:cut], ticks_h[:cut], T, cand, mode)
            got = cnt.cpu().numpy()
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (mode, dispatch, cut, bad[:5], got[bad[:5]], want[bad[:5]])
            prev = cut
    finally:
        ctx.set_param(fe.PARAM_TYPE_DISPATCH, 1)
    return cnt.cpu().numpy(), last.cpu().numpy()


@pytest.mark.parametrize("mode", [RELAXED, EXACT])
def test_partitions_match_whole_stream(ctx, fe, mode):
    rng = np.random.default_rng(31 + mode)
    T = 10
    ids_h, ticks_h = _stream(rng, 30_000, T, 20)
    cand = _cands(rng, T)
    n = ids_h.size
    cuts = sorted(set([0, 1, 2, 64, 65, 1000, 1001, 1001, 7777, 20_000, n - 1, n]
                      + rng.integers(0, n, 12).tolist()))
    banner("resume: mode=%d, %d candidates, %d partitions" % (mode, cand["M"], len(cuts)))
    for dispatch in (1, 0):
        cnt, last = _run(ctx, fe, ids_h, ticks_h, T, cand, mode, cuts, dispatch)
    # the carried index is the last completion: for a sample of candidates,
    # the count over [0, last] is the total and over [0, last) one less
    pick = rng.choice(cand["M"], 24, replace=False)
    for m in pick:
        one = {k: (v[m:m + 1] if isinstance(v, np.ndarray) else v) for k, v in cand.items()}
        one["M"] = 1
        if cnt[m] == 0:
            assert last[m] == -1, m
            continue
        L = int(last[m])
        upto = oracle_counts(ids_h[:L + 1], ticks_h[:L + 1], T, one, mode)[0]
        below = oracle_counts(ids_h[:L], ticks_h[:L], T, one, mode)[0]
        assert upto == cnt[m] and below == cnt[m] - 1, (m, L, upto, below, cnt[m])


def test_resume_on_mining_partitions(ctx, fe):
    # the mining workload's level-3 candidate tiles, counted in 8 partitions
    s = synth.config_mining(duration_s=120.0)
    rng = np.random.default_rng(5)
    eps = synth.random_episodes(rng, 3000, s["num_types"], 3, s["intervals"])
    cand = synth.pack(eps)
    n = s["ids"].size
    cuts = [int(n * k / 8) for k in range(1, 9)]
    banner("resume on mining stream: n=%d, %d candidates" % (n, cand["M"]))
    for mode in (RELAXED, EXACT):
        _run(ctx, fe, s["ids"], s["ticks"], s["num_types"], cand, mode, cuts, 1)


def test_resume_errors(ctx, fe):
    t = ctx.torch
    rng = np.random.default_rng(2)
    ids_h, ticks_h = _stream(rng, 100, 4, 5)
    ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
    cand = synth.pack([((0, 1), (0,), (10,))])
    cnt = t.zeros(1, dtype=t.int32, device=ctx.device)
    last = t.full((1,), -1, dtype=t.int32, device=ctx.device)
    with pytest.raises(fe.FeError):
        ctx.count_resume(ids, ticks, 4, cand, EXACT, 101, cnt, last)
    with pytest.raises(fe.FeError):
        ctx.count_resume(ids, ticks, 4, cand, EXACT, -1, cnt, last)
    # from == n: nothing new, carry unchanged
    ctx.count_resume(ids, ticks, 4, cand, EXACT, 100, cnt, last)
    assert int(cnt.item()) == 0 and int(last.item()) == -1
