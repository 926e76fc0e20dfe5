"""Parity at full workload sizes, in the launch configuration the benchmark
uses: sampled outputs checked one by one against the oracle, and invariants
that hold for every candidate."""
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


def _sub(cand, idx):
    return {"types": cand["types"][idx], "len": cand["len"][idx], "lo": cand["lo"][idx],
            "hi": cand["hi"][idx], "nmax": cand["nmax"], "M": len(idx)}


def test_large_array_two_pass_sampled(ctx):
    s = synth.config_large()
    n = s["ids"].size
    banner("large: n=%d theta=%d" % (n, s["theta"]))
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    rng = np.random.default_rng(8)
    for N, cand in s["candidate_sets"].items():
        up, ex, ns = ctx.count_two_pass(ids, ticks, s["num_types"], cand, s["theta"])
        up, ex = up.cpu().numpy(), ex.cpu().numpy()
        kept = up >= s["theta"]
        assert int(ns.item()) == int(kept.sum())
        assert ((ex == -1) == ~kept).all()
        assert (up[kept] >= ex[kept]).all()          # Theorem of Sec. 5.3.2
        n_planted = sum(len(synth.sub_episodes(c, N)) for c in s["cascades"])
        idx = np.unique(np.concatenate([np.arange(min(n_planted, cand["M"])),
                                        rng.choice(cand["M"], 250, replace=False)]))
        sub = _sub(cand, idx)
        wu, we = oracle.two_pass(s["ids"], s["ticks"], s["num_types"], sub["types"], sub["len"],
                                 sub["lo"], sub["hi"], s["theta"], projection=True)
        assert (up[idx] == wu).all(), N
        assert (ex[idx] == we).all(), N
        banner("N=%d: %d survivors, %d frequent, %d checked" % (
            N, int(kept.sum()), int((ex >= s["theta"]).sum()), idx.size))


def test_mining_workload_sampled(ctx):
    s = synth.config_mining()
    theta = s["theta"]
    banner("mining: n=%d theta=%d" % (s["ids"].size, theta))
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    res = ctx.mine(ids, ticks, s["num_types"], s["intervals"], theta, 6)
    F = {}
    for lv in res:
        F[lv["level"]] = {(tuple(t), tuple(a), tuple(b)): (int(u), int(x))
                          for t, a, b, u, x in zip(lv["types"], lv["lo"], lv["hi"], lv["upper"],
                                                   lv["exact"])}
    # level 1 is the histogram
    hist = np.bincount(s["ids"], minlength=s["num_types"])
    assert set(k[0][0] for k in F[1]) == set(np.nonzero(hist >= theta)[0].tolist())
    # planted cascades are found with their planted intervals
    for c in s["cascades"]:
        if c["firings"] < theta:
            continue
        for L in range(2, min(len(c["neurons"]), 6) + 1):
            for ep in synth.sub_episodes(c, L):
                assert ep in F[L], ep
    rng = np.random.default_rng(21)
    for L in range(2, 5):
        # random episodes: frequent according to the oracle <=> reported frequent
        eps = synth.random_episodes(rng, 300, s["num_types"], L, s["intervals"])
        # plus a sample of the reported frequent set
        rep = list(F[L].keys())
        pick = rng.choice(len(rep), min(100, len(rep)), replace=False)
        eps += [rep[i] for i in pick]
        pk = synth.pack(eps)
        wu, we = oracle.two_pass(s["ids"], s["ticks"], s["num_types"], pk["types"], pk["len"],
                                 pk["lo"], pk["hi"], theta, projection=True)
        for e, u, x in zip(eps, wu, we):
            freq = x >= theta
            assert (e in F[L]) == freq, (L, e, u, x)
            if freq:
                assert F[L][e] == (int(u), int(x)), (L, e)
        banner("level %d: %d frequent reported, %d checked" % (L, len(F[L]), len(eps)))
    # anti-monotonicity of the reported sets
    for L in range(3, max(F) + 1):
        for (t, a, b), (u, x) in F[L].items():
            assert (t[:-1], a[:-1], b[:-1]) in F[L - 1] and (t[1:], a[1:], b[1:]) in F[L - 1]
