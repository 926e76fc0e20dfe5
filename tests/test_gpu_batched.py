"""GPU parity of the batched path: every recording's relaxed and exact
counts from one planned batch (persistent launches replayed from captured
graphs) equal the oracle's and the same recording counted alone."""
import numpy as np
import pytest

import oracle
from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _small_batch(R=6, seed=3):
    recs = synth.config_batched(R=R, n_lo=2e3, n_hi=6e4, m_lo=50, m_hi=600, tag=41 + seed)
    return recs


def _want(rec):
    c = rec["candidates"]
    return oracle.two_pass(rec["ids"], rec["ticks"], rec["num_types"], c["types"], c["len"],
                           c["lo"], c["hi"], rec["theta"], projection=True)


def _dev(ctx, recs):
    out = []
    for r in recs:
        ids, ticks = ctx.stream_tensors(r["ids"], r["ticks"])
        out.append({"ids": ids, "ticks": ticks, "num_types": r["num_types"],
                    "cand": ctx.cand_tensors(r["candidates"]), "theta": r["theta"]})
    return out


@pytest.mark.parametrize("seg_events,wpb", [(256, 4), (2048, 1), (2048, 8), (32768, 2)])
def test_batch_matches_oracle(ctx, fe, seg_events, wpb):
    recs = _small_batch()
    banner("batch of %d, seg_events=%d, waves_per_block=%d" % (len(recs), seg_events, wpb))
    dev = _dev(ctx, recs)
    b = fe.Batch(ctx, dev)
    b.set_tuning(seg_events, 8, wpb)
    assert b.tuning()["waves_per_block"] == wpb
    for rep in range(2):  # replays must give the same result
        b.run()
        ctx.sync()
        for r, rec in enumerate(recs):
            wu, we = _want(rec)
            assert (b.upper[r].cpu().numpy() == wu).all(), (rep, r)
            assert (b.exact[r].cpu().numpy() == we).all(), (rep, r)
    b.close()


def test_batch_equals_alone_and_autotune(ctx, fe):
    recs = _small_batch(R=5, seed=9)
    dev = _dev(ctx, recs)
    b = fe.Batch(ctx, dev)
    t = b.autotune(reps=1)
    banner("autotuned %s" % t)
    assert t["seg_events"] > 0 and t["waves_per_cu"] > 0 and t["waves_per_block"] in (2, 4, 8)
    b.run()
    ctx.sync()
    for r, d in enumerate(dev):
        up, ex, ns = ctx.count_two_pass(d["ids"], d["ticks"], d["num_types"], d["cand"], d["theta"])
        assert (b.upper[r].cpu().numpy() == up.cpu().numpy()).all(), r
        assert (b.exact[r].cpu().numpy() == ex.cpu().numpy()).all(), r
    b.close()


def test_tuning_rejects_bad_shapes(ctx, fe):
    b = fe.Batch(ctx, _dev(ctx, _small_batch(R=2, seed=5)))
    for seg, wp, wb in [(128, 8, 4), (4096, 0, 4), (4096, 8, 3), (4096, 8, 16)]:
        with pytest.raises(fe.FeError):
            b.set_tuning(seg, wp, wb)
    b.set_tuning(4096, 8)  # 0 waves per block: the default
    assert b.tuning()["waves_per_block"] == 4
    b.close()
