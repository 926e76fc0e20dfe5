"""Parity at full workload sizes, in the launch configurations the benchmark
uses, element by element against the oracle.

The oracle needs minutes to an hour of CPU time per workload at these sizes,
so its outputs are stored under tests/golden/ by a committed script that
calls only the seeded input generators and oracle/
(tests/golden/make_fullsize.py, which also states each sample).  Each test
regenerates the inputs, checks their fingerprint against the stored one
(so the stored values belong to these inputs), and compares:

* mining workload (64 neurons x 20 Hz x 780 s, levels 2-6): the level list,
  candidate and survivor numbers, and the whole frequent set with its counts
  at every level; the counts of every candidate of levels 2, 5 and 6; the
  counts of the stated seeded sample of levels 3 and 4 (256 consecutive
  tiles, 20000 random candidates, every planted sub-episode);
* large array (about 1.1e7 events, 256 neurons): both 1e5-candidate sets,
  both counters, every candidate;
* batched (64 recordings, 727774 candidates): every candidate's two-pass
  result from the autotuned batch;
* served (the full 60 s trace, about 12000 requests): every request served
  through the continuous-batching server, and a seeded 5% sample compared
  with the oracle by SHA-256 of the whole per-request result arrays.

Two-pass outputs are compared as Algorithm 4 defines them: upper = the
relaxed count, exact = the exact count where upper >= theta, else -1."""
import hashlib
import os

import numpy as np
import pytest

from paper_0905_2200_amd import synth
from tests.gpu_util import banner, have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(np.asarray(a), dtype="<i4").tobytes())
    return h.hexdigest()


def _gold(name):
    p = os.path.join(GOLD, name)
    if not os.path.exists(p):
        pytest.skip("%s not written yet (python -m tests.golden.make_fullsize)" % name)
    return np.load(p)


def _two_pass(upper, exact_all, theta):
    return np.where(upper >= theta, exact_all, -1)


@pytest.fixture(scope="module")
def fe():
    from paper_0905_2200_amd import fe as fe_mod
    return fe_mod


@pytest.fixture(scope="module")
def ctx(fe):
    c = fe.Context(0)
    yield c
    c.close()


def _hash_rows(rows):
    """64-bit polynomial hash of each int row (wrapping uint64 arithmetic)."""
    h = np.zeros(rows.shape[0], np.uint64)
    mul = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        for k in range(rows.shape[1]):
            h = h * mul + (rows[:, k].astype(np.int64).astype(np.uint64) + np.uint64(k + 1))
    return h


def _locate(big, small):
    """Index in big of each row of small; every row must be present."""
    hb, hs = _hash_rows(big), _hash_rows(small)
    order = np.argsort(hb, kind="stable")
    pos = np.searchsorted(hb[order], hs)
    assert (pos < hb.size).all(), "a candidate is missing"
    idx = order[pos]
    assert (big[idx] == small).all(), "a candidate is missing"
    return idx


def _rows(types, lo, hi):
    return np.concatenate([np.asarray(types), np.asarray(lo), np.asarray(hi)],
                          axis=1).astype(np.int64)


def test_mining_workload_full(ctx, fe):
    s = synth.config_mining()
    g = _gold("fullsize_mining.npz")
    fp = digest(s["ids"], s["ticks"], np.asarray(s["intervals"]), [s["theta"]])
    assert str(g["fingerprint"]) == fp, "the mining workload changed since its golden values"
    theta = s["theta"]
    banner("mining full: n=%d theta=%d" % (s["ids"].size, theta))
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    ctx.set_param(fe.PARAM_KEEP_CANDIDATES, 1)
    try:
        res = ctx.mine(ids, ticks, s["num_types"], s["intervals"], theta, 6)
    finally:
        ctx.set_param(fe.PARAM_KEEP_CANDIDATES, 0)
    # the stored levels (the golden file is written level by level; when it
    # is complete it also fixes the level list)
    done = g["levels_done"].tolist()
    if bool(g["complete"]):
        assert [lv["level"] for lv in res] == g["levels"].tolist()
    assert set(done) <= set(lv["level"] for lv in res) and {1, 2} <= set(done)
    for lv in res:
        L = lv["level"]
        if L not in done:
            continue
        banner("level %d: %d candidates, %d passes" % (L, lv["n_candidates"], lv["passes"]))
        assert lv["n_candidates"] == int(g["n_candidates_%d" % L]), L
        two = L >= 2 and lv["passes"] == 2
        if L >= 2:
            want_surv = int(g["n_survivors_%d" % L]) if two else lv["n_candidates"]
            assert lv["n_survivors"] == want_surv, L
        # the whole frequent set with its counts
        got = _rows(lv["types"], lv["lo"], lv["hi"])
        want = _rows(g["F_types_%d" % L], g["F_lo_%d" % L], g["F_hi_%d" % L])
        assert got.shape == want.shape, (L, got.shape, want.shape)
        idx = _locate(got, want)
        assert (np.asarray(lv["exact"])[idx] == g["F_exact_%d" % L]).all(), L
        if two or L == 1:
            assert (np.asarray(lv["upper"])[idx] == g["F_upper_%d" % L]).all(), L
        if L == 1:
            continue
        # per candidate: every one (levels 2, 5, 6) or the stated sample (3, 4)
        rows = _rows(lv["all_types"], lv["all_lo"], lv["all_hi"])
        pre = "all_" if ("all_types_%d" % L) in g.files else "s_"
        want_rows = _rows(g[pre + "types_%d" % L], g[pre + "lo_%d" % L], g[pre + "hi_%d" % L])
        if pre == "all_":
            assert want_rows.shape[0] == rows.shape[0]
        idx = _locate(rows, want_rows)
        up_w, ex_w = g[pre + "upper_%d" % L], g[pre + "exact_%d" % L]
        if two:
            assert (lv["all_upper"][idx] == up_w).all(), L
            assert (lv["all_exact"][idx] == _two_pass(up_w, ex_w, theta)).all(), L
        else:
            assert (lv["all_upper"] == -1).all(), L
            assert (lv["all_exact"][idx] == ex_w).all(), L
        banner("level %d: %d frequent, %d candidates compared" % (L, lv["n_frequent"], idx.size))


def test_large_array_full(ctx):
    s = synth.config_large()
    g = _gold("fullsize_large.npz")
    assert str(g["fingerprint"]) == digest(s["ids"], s["ticks"], [s["theta"]])
    theta = s["theta"]
    banner("large full: n=%d theta=%d" % (s["ids"].size, theta))
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    for N, cand in s["candidate_sets"].items():
        assert str(g["cand_fp_%d" % N]) == digest(cand["types"], cand["len"], cand["lo"],
                                                  cand["hi"])
        up_w, ex_w = g["upper_%d" % N], g["exact_%d" % N]
        up, ex, ns = ctx.count_two_pass(ids, ticks, s["num_types"], cand, theta)
        up, ex = up.cpu().numpy(), ex.cpu().numpy()
        assert (up == up_w).all(), (N, np.nonzero(up != up_w)[0][:5])
        assert (ex == _two_pass(up_w, ex_w, theta)).all(), N
        assert int(ns.item()) == int((up_w >= theta).sum())
        exact_all = ctx.count(ids, ticks, s["num_types"], cand, 0).cpu().numpy()
        assert (exact_all == ex_w).all(), N
        banner("N=%d: %d candidates, %d survivors, %d frequent" % (
            N, cand["M"], int((up_w >= theta).sum()), int((ex_w >= theta).sum())))


def test_batched_full(ctx, fe):
    recs = synth.config_batched()
    g = _gold("fullsize_batched.npz")
    fps = "".join(digest(r["ids"], r["ticks"], [r["theta"]]) +
                  digest(r["candidates"]["types"], r["candidates"]["len"], r["candidates"]["lo"],
                         r["candidates"]["hi"]) for r in recs)
    assert str(g["fingerprint"]) == digest(np.frombuffer(fps.encode(), np.uint8))
    banner("batched full: %d recordings, %d candidates" % (len(recs), int(g["offsets"][-1])))
    dev = []
    for r in recs:
        ids, ticks = ctx.stream_tensors(r["ids"], r["ticks"])
        dev.append({"ids": ids, "ticks": ticks, "num_types": r["num_types"],
                    "cand": ctx.cand_tensors(r["candidates"]), "theta": r["theta"]})
    b = fe.Batch(ctx, dev)
    tun = b.autotune(reps=1)
    banner("autotuned %s" % tun)
    for rep in range(2):
        b.run()
        ctx.sync()
        off = g["offsets"]
        for k, r in enumerate(recs):
            up_w, ex_w = g["upper"][off[k]:off[k + 1]], g["exact"][off[k]:off[k + 1]]
            assert (b.upper[k].cpu().numpy() == up_w).all(), (rep, k)
            assert (b.exact[k].cpu().numpy() == _two_pass(up_w, ex_w, r["theta"])).all(), (rep, k)
    b.close()


def test_served_trace_full(ctx, fe):
    sv = synth.config_served(trace_s=60.0)
    reqs, arrays, cand = sv["requests"], sv["arrays"], sv["candidates"]
    g = _gold("fullsize_served.npz")
    fp = digest(np.array([[r["array"], r["t_begin"], r["t_end"], r["theta"]] for r in reqs]),
                *[np.concatenate([a["ids"], a["ticks"]]) for a in arrays],
                cand["types"], cand["len"], cand["lo"], cand["hi"])
    assert str(g["fingerprint"]) == fp
    sample = {int(i): k for k, i in enumerate(g["sample"])}
    assert len(sample) >= 0.05 * len(reqs)
    banner("served full trace: %d requests, %d sampled" % (len(reqs), len(sample)))
    server = fe.Server(ctx, cand, [a["num_types"] for a in arrays],
                       capacity=max(a["ids"].size for a in arrays) + 16, hbm_budget=16 << 30,
                       max_inflight=3, max_round=64)
    for k, a in enumerate(arrays):
        server.append(k, a["ids"], a["ticks"])
    tickets = [server.submit(r["array"], r["t_begin"], r["t_end"], r["theta"]) for r in reqs]
    checked = 0
    for i, t in enumerate(tickets):
        k = sample.get(i)
        res = server.wait(t, copy=k is not None)
        assert res["status"] == fe.FE_OK, i
        if k is not None:
            assert res["n_events"] == int(g["n_events"][k]), i
            assert res["n_survivors"] == int(g["n_survivors"][k]), i
            assert res["n_frequent"] == int(g["n_frequent"][k]), i
            assert digest(res["upper"]) == str(g["upper_sha"][k]), i
            assert digest(res["exact"]) == str(g["exact_sha"][k]), i
            checked += 1
        server.release(t)
        if i % 2000 == 0:
            banner("served: %d of %d done" % (i, len(reqs)))
    st = server.stats()
    server.close()
    assert checked == len(sample)
    banner("served: %d rounds, largest %d" % (st["rounds"], st["largest_round"]))
