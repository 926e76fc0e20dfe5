"""GPU tests of the serving path: every request's counts equal the oracle's
on its window and the same window counted alone, whatever the mix of
requests sharing its round; admission by device-memory footprint."""
import time

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


@pytest.fixture(scope="module")
def served():
    return synth.config_served(n_arrays=4, trace_s=2.0, preroll_s=8.0, M=1500, rate_req=40.0,
                               win_lo_s=0.5, win_hi_s=8.0, tag=77)


def _window(arr, t0, t1):
    a = np.searchsorted(arr["ticks"], t0, "left")
    b = np.searchsorted(arr["ticks"], t1, "left")
    return arr["ids"][a:b], arr["ticks"][a:b]


def _server(fe, ctx, sv, **kw):
    s = fe.Server(ctx, sv["candidates"], [a["num_types"] for a in sv["arrays"]],
                  capacity=max(a["ids"].size for a in sv["arrays"]) + 16, **kw)
    for k, a in enumerate(sv["arrays"]):
        s.append(k, a["ids"], a["ticks"])
    return s


def test_served_requests_match_oracle_and_alone(fe, ctx, served):
    sv = served
    reqs = sv["requests"]
    banner("served: %d requests, M=%d" % (len(reqs), sv["candidates"]["M"]))
    s = _server(fe, ctx, sv, hbm_budget=1 << 30, max_inflight=3, max_round=6)
    tickets = [s.submit(r["array"], r["t_begin"], r["t_end"], r["theta"]) for r in reqs]
    res = [s.wait(t) for t in tickets]
    st = s.stats()
    banner("stats %s" % st)
    assert st["completed"] == len(reqs) and st["rounds"] < len(reqs)
    c = sv["candidates"]
    dc = ctx.cand_tensors(c)
    for k, (r, out) in enumerate(zip(reqs, res)):
        assert out["status"] == 0
        ids, ticks = _window(sv["arrays"][r["array"]], r["t_begin"], r["t_end"])
        assert out["n_events"] == ids.size
        if k % 3 == 0:
            wu, we = oracle.two_pass(ids, ticks, sv["arrays"][r["array"]]["num_types"], c["types"],
                                     c["len"], c["lo"], c["hi"], r["theta"], projection=True)
            assert (out["upper"] == wu).all(), k
            assert (out["exact"] == we).all(), k
        # the same window counted alone
        di, dt = ctx.stream_tensors(ids, ticks)
        up, ex, ns = ctx.count_two_pass(di, dt, sv["arrays"][r["array"]]["num_types"], dc,
                                        r["theta"])
        assert (out["upper"] == up.cpu().numpy()).all(), k
        assert (out["exact"] == ex.cpu().numpy()).all(), k
        assert out["n_survivors"] == int(ns.item())
    for t in tickets:
        s.release(t)
    s.close()


def test_tiny_budget_one_request_per_round_and_rejection(fe, ctx, served):
    sv = served
    reqs = sv["requests"][:12]
    s = _server(fe, ctx, sv, hbm_budget=1, max_inflight=1, max_round=8)
    tickets = [s.submit(r["array"], r["t_begin"], r["t_end"], r["theta"]) for r in reqs]
    res = [s.wait(t) for t in tickets]
    # each request alone exceeds a 1-byte budget: all are rejected
    assert all(o["status"] == 2 for o in res)
    s.close()
    # a budget that fits one request at a time: one request per round
    s = _server(fe, ctx, sv, hbm_budget=600 << 10, max_inflight=1, max_round=8)
    tickets = [s.submit(r["array"], r["t_begin"], r["t_end"], r["theta"]) for r in reqs]
    res = [s.wait(t) for t in tickets]
    assert all(o["status"] == 0 for o in res)
    st = s.stats()
    banner("tiny budget stats %s" % st)
    c = sv["candidates"]
    for r, out in zip(reqs, res):
        ids, ticks = _window(sv["arrays"][r["array"]], r["t_begin"], r["t_end"])
        wu, we = oracle.two_pass(ids, ticks, sv["arrays"][r["array"]]["num_types"], c["types"],
                                 c["len"], c["lo"], c["hi"], r["theta"], projection=True)
        assert (out["exact"] == we).all()
    s.close()


def test_append_errors(fe, ctx, served):
    sv = served
    s = _server(fe, ctx, sv, hbm_budget=1 << 28, max_inflight=1, max_round=4)
    with pytest.raises(fe.FeError) as e:
        s.append(0, [1, 2], [5, 4])
    assert e.value.code in (fe.FE_EUNSORTED,)
    with pytest.raises(fe.FeError) as e:
        s.append(0, [100000], [sv["arrays"][0]["ticks"][-1] + 5])
    assert e.value.code == fe.FE_ERANGE
    s.close()
