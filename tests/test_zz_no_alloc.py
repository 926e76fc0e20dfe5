"""fe_count_noalloc (fe_count whose workspace is the library's fixed device
scratch) gives fe_count's results, through the C ABI, on two calls in a row,
the second with a smaller input; the fixed scratch keeps the first call's
contents, so this also checks that everything that must start cleared is
cleared.  Oversized inputs are refused before any work is enqueued."""
import numpy as np
import pytest

from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu, oracle_counts

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

EXACT, RELAXED = 0, 1
IVS = [(0, 50), (50, 100), (100, 200), (190, 200)]   # the last is a deep-class hop


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _case(seed, n, T, M, nmax):
    rng = np.random.default_rng(seed)
    ids = rng.integers(0, T, size=n).astype(np.int32)
    ticks = np.cumsum(rng.integers(0, 9, size=n)).astype(np.int32)
    eps = synth.random_episodes(rng, M, T, nmax, IVS, n_min=1)
    for last in range(T):           # a shared-prefix run
        eps.append(((1, 2, last), (0, 50), (50, 100)))
    return ids, ticks, synth.pack(eps)


@pytest.mark.parametrize("P", [0, 64])
def test_noalloc_equals_fe_count_twice(ctx, P):
    t = ctx.torch
    ctx.set_param(0, P)
    try:
        for k, (seed, n, T, M, nmax) in enumerate([(1, 60000, 8, 3000, 6),
                                                   (2, 9000, 5, 700, 4)]):
            ids_h, ticks_h, cand = _case(seed, n, T, M, nmax)
            banner("noalloc call %d: n=%d M=%d P=%d" % (k, n, cand["M"], P))
            ids, ticks = ctx.stream_tensors(ids_h, ticks_h)
            cd = ctx.cand_tensors(cand)
            for mode in (EXACT, RELAXED):
                out = t.full((cand["M"],), -7, dtype=t.int32, device=ctx.device)
                got = ctx.count_noalloc(ids, ticks, T, cd, mode, out).cpu().numpy()
                ref = ctx.count(ids, ticks, T, cd, mode).cpu().numpy()
                assert (got == ref).all(), (k, mode, np.nonzero(got != ref)[0][:5])
                want = oracle_counts(ids_h, ticks_h, T, cand, mode)
                assert (got == want).all(), (k, mode)
    finally:
        ctx.set_param(0, 0)


def test_noalloc_refuses_oversized_input(ctx, fe):
    t = ctx.torch
    M = 3_000_000   # about 4 B + 88 B per candidate of 8 nodes: beyond 64 MiB
    cand = {"types": t.zeros((M, 8), dtype=t.int32, device=ctx.device),
            "len": t.ones(M, dtype=t.int32, device=ctx.device),
            "lo": t.zeros((M, 7), dtype=t.int32, device=ctx.device),
            "hi": t.ones((M, 7), dtype=t.int32, device=ctx.device), "nmax": 8, "M": M}
    ids, ticks = ctx.stream_tensors(np.zeros(10, np.int32), np.arange(10, dtype=np.int32))
    out = t.empty(M, dtype=t.int32, device=ctx.device)
    with pytest.raises(fe.FeError) as e:
        ctx.count_noalloc(ids, ticks, 1, cand, EXACT, out)
    assert e.value.code == fe.FE_ENOMEM
    # the context still works
    small = synth.pack([((0, 0), (0,), (3,))])
    assert ctx.count_noalloc(ids, ticks, 1, small, EXACT,
                             t.empty(1, dtype=t.int32, device=ctx.device))[0].item() == 5
