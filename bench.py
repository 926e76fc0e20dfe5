#!/usr/bin/env python3
"""Throughput benchmark of the episode-counting hot path on one MI355X.

Default line (one JSON line on stdout): the mining workload -- 64 neurons
firing at 20 Hz for 780 s (about 1.05M events, int32 ids and 0.1 ms int32
ticks) with eight planted cascades of 3-6 nodes, hop intervals
{(0,5], (5,10], (10,20]} ms, levels 2-6, threshold 0.5 Hz x 780 s = 390.
One step = one complete level-wise mining run (Problem 1): each level is
generated on the host and counted on the GPU (MapConcatenate Map and
Concatenate kernels; two-pass elimination, Algorithm 4, where the library's
per-level rule finds that the relaxed pass pays for itself).

Metric: candidate-episode x events per second, a step's work being
sum over levels >= 2 of (candidates x events): every candidate counted
against every event once, however many passes the library takes; also the
time per mined set (= per step).  The stream is resident in HBM before the
timed region.  The same line carries, as sub-objects, the batched workload
(one planned batch against one fe_count_two_pass per recording), the served
workload (continuous batching against one request per launch, p50/p99, and
a run whose device-memory budget binds), the large-array workload, the
roofline of the dominant kernel and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_EE = 8  # one int32 id + one int32 tick per event per candidate machine
# instruction issue: 256 CUs x 4 SIMDs, 2.4 GHz, one wave64 VALU (or SALU)
# instruction per SIMD every 4 cycles
ISSUE_PEAK_G = 1024 * 2.4 / 4  # 614.4 G wave-instructions/s
MAP_SOURCES = ["paper_0905_2200_amd/csrc/fe_map.h"] + [
    "paper_0905_2200_amd/csrc/fe_map_n%d.hip" % n for n in range(1, 9)]
COUNTERS = os.path.join(ROOT, "profiles", "map_counters.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def map_source_hash():
    h = hashlib.sha256()
    for p in MAP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters_for(kernel):
    """Per-launch rocprofv3 counters of `kernel` on this workload from the
    committed summary, if they were taken on the current Map sources."""
    if not os.path.exists(COUNTERS):
        return None
    try:
        d = json.load(open(COUNTERS))
    except Exception:
        return None
    if d.get("map_source_hash") != map_source_hash():
        return None
    return d.get("kernels", {}).get(kernel)


def pct(a, q):
    import numpy as np
    return round(float(np.percentile(a, q)), 2) if len(a) else None


# ---------------------------------------------------------------- mining
def bench_mining(args, fe, synth, torch):
    import numpy as np
    s = synth.config_mining(duration_s=args.duration_s)
    n = int(s["ids"].size)
    theta, intervals = s["theta"], s["intervals"]
    log("workload: %s; n=%d theta=%d" % (s["name"], n, theta))
    ctx = fe.Context(0)
    ctx.set_param(fe.PARAM_TYPE_DISPATCH, args.type_dispatch)
    ctx.set_param(fe.PARAM_SHARED_LISTS, args.shared_lists)
    if args.elimination is not None:
        ctx.set_param(fe.PARAM_ELIMINATION, args.elimination)
    if args.host_tiling is not None:
        ctx.set_param(fe.PARAM_HOST_TILING, args.host_tiling)
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    torch.cuda.synchronize()
    if args.calib_copy_mib:
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        return ctx.mine(ids, ticks, s["num_types"], intervals, theta, args.max_level)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        res = step()
        torch.cuda.synchronize()
        log("warmup step %d: %.3f s" % (w, time.perf_counter() - t0))
    ctx.set_param(fe.PARAM_TIMING, 1)
    ctx.reset_kernel_stats()
    times = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        res = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log("step %d: %.3f s" % (len(times) - 1, times[-1]))
    t_total = time.perf_counter() - t_start
    kst = ctx.kernel_stats()
    ctx.set_param(fe.PARAM_TIMING, 0)
    ctx.close()

    ee_step = sum(lv["n_candidates"] * n for lv in res if lv["level"] >= 2)
    counted = sum((lv["n_candidates"] if lv["passes"] == 1 else
                   lv["n_candidates"] + lv["n_survivors"]) * n for lv in res if lv["level"] >= 2)
    for lv in res:
        log("level %d: candidates %d survivors %d frequent %d passes %d sample %d/%d gen %.1f ms "
            "count %.1f ms" % (lv["level"], lv["n_candidates"], lv["n_survivors"],
                               lv["n_frequent"], lv["passes"], lv["sample_kept"], lv["sample_n"],
                               lv["gen_ms"], lv["count_ms"]))
    host = {k: v for k, v in kst.items() if k.startswith("host_")}
    kst = {k: v for k, v in kst.items() if not k.startswith("host_")}
    tot_kms = sum(v["total_ms"] for v in kst.values())
    for k, v in sorted(kst.items(), key=lambda kv: -kv[1]["total_ms"]):
        log("kernel %-24s launches %5d total %9.2f ms (%.1f%%) ee %.3e" % (
            k, v["launches"], v["total_ms"], 100 * v["total_ms"] / max(tot_kms, 1e-9), v["ee"]))
    for k, v in sorted(host.items(), key=lambda kv: -kv[1]["total_ms"]):
        log("host phase %-20s calls %5d total %9.2f ms" % (k[5:], v["launches"], v["total_ms"]))

    maps = {k: v for k, v in kst.items() if k.startswith("map_") and v["total_ms"] > 0}
    dom = max(maps.items(), key=lambda kv: kv[1]["total_ms"]) if maps else None
    roofline = stream_eq = dram = None
    if dom:
        name, v = dom
        t_launch = v["total_ms"] / v["launches"] * 1e-3
        ee_launch = v["ee"] / v["launches"]
        cnt = counters_for(name)
        issued = None
        if cnt:
            issued = max(cnt["valu_per_launch"], cnt["salu_per_launch"])
        achieved = issued / t_launch / 1e9 if issued else None
        roofline = {
            "bound": "alu", "achieved": round(achieved, 2) if achieved else None,
            "peak": ISSUE_PEAK_G, "unit": "G wave-instr/s",
            "frac": round(achieved / ISSUE_PEAK_G, 4) if achieved else None,
            "traffic": cnt.get("hbm_bytes_per_launch") if cnt else None,
            "kernel": name, "avg_launch_ms": round(t_launch * 1e3, 4), "launches": v["launches"],
            "derivation": ("instruction issue of the dominant kernel: max(VALU, SALU) wave64 "
                           "instructions per launch (rocprofv3 SQ_INSTS_VALU, SQ_INSTS_SALU, "
                           "profiles/map_counters.json) / the launch's HIP-event duration; peak "
                           "= 1024 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction")}
        stream_eq = {"bytes_per_ee": BYTES_PER_EE, "ee_per_launch": ee_launch,
                     "achieved_GBs": round(BYTES_PER_EE * ee_launch / t_launch / 1e9, 1),
                     "peak_GBs": HBM_PEAK_GBS,
                     "frac": round(BYTES_PER_EE * ee_launch / t_launch / 1e9 / HBM_PEAK_GBS, 3),
                     "note": "8 B per candidate-event as if every machine read every event; "
                             "not DRAM traffic"}
        if cnt and cnt.get("hbm_bytes_per_launch"):
            gbs = cnt["hbm_bytes_per_launch"] / t_launch / 1e9
            dram = {"beyond_l2_bytes_per_launch": cnt["hbm_bytes_per_launch"],
                    "achieved_GBs": round(gbs, 1), "peak_GBs": HBM_PEAK_GBS,
                    "frac": round(gbs / HBM_PEAK_GBS, 4)}
    times_ms = sorted(1e3 * t for t in times)
    return {
        "value": float("%.5g" % (ee_step * args.steps / t_total)),
        "ms_per_step": round(1e3 * t_total / args.steps, 2),
        "p50_ms": pct(times_ms, 50), "p99_ms": pct(times_ms, 99),
        "config": {"workload": "level-wise mining of one stream, levels 2-%d" % args.max_level,
                   "neurons": s["num_types"], "rate_hz": 20, "duration_s": args.duration_s,
                   "n_events": n, "theta": theta, "intervals_ticks": intervals,
                   "ee_per_step": ee_step, "ee_counted_per_step": counted,
                   "levels": [{k: lv[k] for k in ("level", "n_candidates", "n_survivors",
                                                   "n_frequent", "passes", "sample_n",
                                                   "sample_kept")} for lv in res]},
        "roofline": roofline, "stream_equivalent": stream_eq, "dram": dram,
        "stream": s}


def cpu_baseline(s, target_s, runs=3):
    """The oracle (as it stands) on a seeded sample of the mining workload's
    level-3 candidates: the oracle's own levels 1 and 2 and its own join give
    the level-3 candidate set; the sample grows until one two-pass run takes
    about target_s; the median of `runs` runs, with the relaxed pass and the
    exact pass (survivors) timed apart.  ee counts each sampled candidate
    against the stream's events once, like the GPU figure."""
    import numpy as np
    import oracle
    from oracle import mine
    ids, ticks, T, theta = s["ids"], s["ticks"], s["num_types"], s["theta"]
    threads = oracle.max_threads()
    hist = np.bincount(ids, minlength=T)
    F1 = np.nonzero(hist >= theta)[0]
    t2, l2, h2 = mine.gen_level2_arrays(F1, s["intervals"])
    up2, ex2 = oracle.two_pass(ids, ticks, T, t2, np.full(t2.shape[0], 2, np.int32), l2, h2,
                               theta, projection=True, nthreads=threads)
    fr = ex2 >= theta
    t3, l3, h3 = mine.gen_next_arrays(*mine.sort_episodes(t2[fr], l2[fr], h2[fr]))
    rng = np.random.default_rng([2, 777])
    perm = rng.permutation(t3.shape[0])
    K = 2000

    def run(k):
        sel = np.sort(perm[:k])
        c = (t3[sel], np.full(k, 3, np.int32), l3[sel], h3[sel])
        t0 = time.perf_counter()
        up = oracle.count(ids, ticks, T, *c, oracle.MODE_RELAXED, projection=True,
                          nthreads=threads)
        t1 = time.perf_counter()
        keep = up >= theta
        oracle.count(ids, ticks, T, c[0][keep], c[1][keep], c[2][keep], c[3][keep],
                     oracle.MODE_EXACT, projection=True, nthreads=threads)
        t2_ = time.perf_counter()
        return t1 - t0, t2_ - t1, int(keep.sum())
    while True:
        a, b, _ = run(K)
        if a + b >= target_s / 2 or K >= t3.shape[0]:
            break
        K = min(t3.shape[0], int(K * max(2.0, target_s / max(a + b, 1e-3) * 0.9)))
    res = [run(K) for _ in range(runs)]
    tot = sorted(a + b for a, b, _ in res)
    med = tot[len(tot) // 2]
    rel = sorted(a for a, _, _ in res)[len(res) // 2]
    exa = sorted(b for _, b, _ in res)[len(res) // 2]
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = ids.size
    return {"value": float("%.4g" % (K * n / med)), "unit": "ee/s", "cores": threads,
            "kind": "oracle",
            "sample": ("two-pass (relaxed pass, elimination, exact pass on the %d survivors) in "
                       "projection mode on a seeded sample of %d of the workload's %d level-3 "
                       "candidates over its %d events; median of %d runs of %.1f s" % (
                           res[0][2], K, t3.shape[0], n, runs, med)),
            "relaxed_pass_ee_per_s": float("%.4g" % (K * n / rel)),
            "exact_pass_s": round(exa, 3), "cpu_model": model}


# ---------------------------------------------------------------- batched
def bench_batched(args, fe, synth, torch, reps=5):
    """64 recordings of uneven length (1e4-1e6 events), 16-256 neurons, each
    with its own 1e3-5e4 candidates of 2-8 nodes; a run = the two-pass count
    of every recording.  Batched: one planned batch (persistent launches, one
    captured graph per episode size, autotuned launch shape).  Plain: one
    fe_count_two_pass call per recording."""
    import numpy as np
    t0 = time.perf_counter()
    recs = synth.config_batched()
    log("batched workload: %d recordings, %d events, %d candidates (%.1f s to generate)" % (
        len(recs), sum(r["ids"].size for r in recs),
        sum(r["candidates"]["M"] for r in recs), time.perf_counter() - t0))
    ctx = fe.Context(0)
    dev = []
    for r in recs:
        ids, ticks = ctx.stream_tensors(r["ids"], r["ticks"])
        dev.append({"ids": ids, "ticks": ticks, "num_types": r["num_types"],
                    "cand": ctx.cand_tensors(r["candidates"]), "theta": r["theta"]})
    torch.cuda.synchronize()

    def plain():
        outs = [ctx.count_two_pass(d["ids"], d["ticks"], d["num_types"], d["cand"], d["theta"])
                for d in dev]
        torch.cuda.synchronize()
        return outs
    outs = plain()
    tp = []
    for _ in range(max(2, reps // 2)):
        t0 = time.perf_counter()
        outs = plain()
        tp.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    b = fe.Batch(ctx, dev)
    t_plan = time.perf_counter() - t0
    tun = b.autotune(reps=2)
    log("batch plan %.2f s; autotuned %s" % (t_plan, tun))
    b.run()
    torch.cuda.synchronize()
    tb = []
    for _ in range(reps):
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    same = all(bool((b.upper[r] == o[0]).all()) and bool((b.exact[r] == o[1]).all())
               for r, o in enumerate(outs))
    ee = sum(d["cand"]["M"] * d["ids"].numel() for d in dev)
    tbm, tpm = float(np.median(tb)), float(np.median(tp))
    b.close()
    ctx.close()
    log("batched %.2f ms, plain %.1f ms" % (1e3 * tbm, 1e3 * tpm))
    return {"value": float("%.5g" % (ee / tbm)), "unit": "ee/s", "ms_per_run": round(1e3 * tbm, 3),
            "p99_ms": pct([1e3 * t for t in tb], 99), "runs": reps,
            "plain_ms_per_run": round(1e3 * tpm, 2),
            "plain_value": float("%.5g" % (ee / tpm)),
            "batched_over_plain": round(tpm / tbm, 2), "identical_results": same,
            "tuning": tun, "plan_s": round(t_plan, 2),
            "config": {"workload": "batched: 64 recordings, two-pass counting",
                       "recordings": len(recs), "events": int(sum(r["ids"].size for r in recs)),
                       "candidates": int(sum(r["candidates"]["M"] for r in recs)),
                       "ee_per_run": ee}}


# ---------------------------------------------------------------- served
def _serve(fe, ctx, sv, reqs, max_inflight, max_round, hbm_budget, copy_every):
    """Replay the trace open-loop (arrivals on the steady clock) through a
    server; returns per-request results, wall time and server stats."""
    import numpy as np
    arrays = sv["arrays"]
    server = fe.Server(ctx, sv["candidates"], [a["num_types"] for a in arrays],
                       capacity=max(a["ids"].size for a in arrays) + 16, hbm_budget=hbm_budget,
                       max_inflight=max_inflight, max_round=max_round)
    ptr = [0] * len(arrays)
    pre = int(sv["preroll_s"] * 10000)
    t_app = [0.0]

    def feed(upto):  # every array's events with tick < upto
        t0 = time.perf_counter()
        for k, a in enumerate(arrays):
            e = int(np.searchsorted(a["ticks"], upto, "left"))
            if e > ptr[k]:
                server.append(k, a["ids"][ptr[k]:e], a["ticks"][ptr[k]:e])
                ptr[k] = e
        t_app[0] += time.perf_counter() - t0
    feed(pre)
    for r in reqs[:4]:  # warm-up before the clock starts
        server.wait(server.submit(r["array"], max(0, pre - 10000), pre, r["theta"]))
    t_app[0] = 0.0
    base = time.monotonic_ns() + 200_000_000
    tickets, late = [], []
    for r in reqs:
        due = base + int(r["arrival_s"] * 1e9)
        feed(pre + int(r["arrival_s"] * 10000) + 1)
        late.append((time.monotonic_ns() - due) / 1e6)
        while time.monotonic_ns() < due:
            pass
        tickets.append(server.submit(r["array"], r["t_begin"], r["t_end"], r["theta"], due))
    done = [server.wait(t, copy=(k % copy_every == 0)) for k, t in enumerate(tickets)]
    stats = server.stats()
    server.close()
    wall = (max(d["done_ns"] for d in done) - base) / 1e9
    stats["submit_late_ms_p50"] = pct(late, 50)
    stats["submit_late_ms_max"] = round(max(late), 2)
    stats["append_s"] = round(t_app[0], 3)
    return done, wall, stats


def bench_served(args, fe, synth, torch):
    """32 simulated arrays (64-256 neurons, 20 Hz) stream events; window
    requests (1-60 s) arrive as a Poisson process at --rate per second; each
    is the two-pass count of 50 000 resident episodes (2-6 nodes) over the
    window.  Three replays of the same open-loop trace: the continuous-
    batching server; one request per launch with the candidates resident
    and pre-tiled (one round of one request at a time); and the server with a
    device-memory budget that binds.  Latency = completion - arrival."""
    import numpy as np
    t0 = time.perf_counter()
    sv = synth.config_served(trace_s=args.trace_s, rate_req=args.rate)
    reqs = sv["requests"]
    log("served workload: %d arrays, %d requests over %.0f s, M=%d (%.1f s to generate)" % (
        len(sv["arrays"]), len(reqs), args.trace_s, sv["candidates"]["M"],
        time.perf_counter() - t0))
    ctx = fe.Context(0)
    M = sv["candidates"]["M"]
    every = 25

    def summary(done, wall, st):
        lat = np.array([(d["done_ns"] - d["arrival_ns"]) / 1e6 for d in done])
        ee = sum(M * d["n_events"] for d in done)
        return {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "wall_s": round(wall, 2),
                "behind_s": round(wall - args.trace_s, 2),
                "ee_per_s": float("%.4g" % (ee / wall)),
                "mean_round_size": round(float(np.mean([d["round_size"] for d in done])), 2),
                "rounds": st["rounds"], "largest_round": st["largest_round"],
                "max_inflight_seen": st["max_inflight_seen"],
                "budget_closed_rounds": st["budget_closed"], "rejected": st["rejected"],
                "submit_late_ms_p50": st["submit_late_ms_p50"],
                "submit_late_ms_max": st["submit_late_ms_max"], "append_s": st["append_s"]}
    big = 16 << 30
    served = _serve(fe, ctx, sv, reqs, args.max_inflight, 64, big, every)
    out = {"served": summary(*served)}
    log("served: %s" % out["served"])
    plain = _serve(fe, ctx, sv, reqs, 1, 1, big, every)
    out["plain_resident"] = summary(*plain)
    log("plain (one request per launch, resident candidates): %s" % out["plain_resident"])
    foot = max(d["footprint"] for d in served[0])
    budget = args.max_inflight * foot
    bound = _serve(fe, ctx, sv, reqs, args.max_inflight, 64, budget, every)
    out["budget_bound"] = summary(*bound)
    out["budget_bound"]["hbm_budget"] = budget
    log("budget-bound (%d bytes): %s" % (budget, out["budget_bound"]))
    same = True
    for k in range(0, len(reqs), every):
        a, b, c = served[0][k], plain[0][k], bound[0][k]
        same &= a["status"] == b["status"] == c["status"] == fe.FE_OK
        same &= bool((a["upper"] == b["upper"]).all() and (a["exact"] == b["exact"]).all())
        same &= bool((a["upper"] == c["upper"]).all() and (a["exact"] == c["exact"]).all())
    ctx.close()
    s = out["served"]
    return {"value": s["ee_per_s"], "unit": "ee/s", "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"],
            **out, "identical_results": same,
            "p99_served_over_plain": round(out["plain_resident"]["p99_ms"] / s["p99_ms"], 2),
            "config": {"workload": "served: 32 arrays, Poisson window requests",
                       "requests": len(reqs), "rate_per_s": args.rate, "trace_s": args.trace_s,
                       "resident_episodes": M, "max_inflight": args.max_inflight}}


# ---------------------------------------------------------------- large
def bench_large(args, fe, synth, torch, reps=3):
    """The large array: 256 neurons, about 1.1e7 events; two sets of 1e5
    candidates (N = 3 and N = 4), each counted by fe_count_two_pass
    (MapConcatenate over the long stream, Algorithm 4)."""
    import numpy as np
    t0 = time.perf_counter()
    s = synth.config_large()
    n = int(s["ids"].size)
    log("large workload: n=%d (%.1f s to generate)" % (n, time.perf_counter() - t0))
    ctx = fe.Context(0)
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    out = {}
    tot_t, tot_ee = 0.0, 0
    for N, c in s["candidate_sets"].items():
        cd = ctx.cand_tensors(c)
        ctx.count_two_pass(ids, ticks, s["num_types"], cd, s["theta"])
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            up, ex, ns = ctx.count_two_pass(ids, ticks, s["num_types"], cd, s["theta"])
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        t = float(np.median(ts))
        out["n%d" % N] = {"ms_per_set": round(1e3 * t, 2), "candidates": c["M"],
                          "survivors": int(ns.item()),
                          "ee_per_s": float("%.4g" % (c["M"] * n / t))}
        tot_t += t
        tot_ee += c["M"] * n
    ctx.close()
    log("large: %s" % out)
    return {"value": float("%.5g" % (tot_ee / tot_t)), "unit": "ee/s",
            "ms_per_two_sets": round(1e3 * tot_t, 2), **out,
            "config": {"workload": "large array: 256 neurons, %d events, two sets of 1e5 "
                                   "candidates (N = 3, 4), two-pass" % n,
                       "n_events": n, "theta": s["theta"]}}


# ---------------------------------------------------------------- streaming
def bench_streaming(args, fe, synth, torch):
    """The mining recording arriving in partitions of --partition-s seconds,
    with every 3-node episode over its 64 neurons x the interval set resident
    (2.36 M candidates); after each partition the exact counts over the
    recording so far are brought up to date by fe_count_resume (carried
    count and last completion per candidate).  Compared with recounting the
    whole prefix with fe_count."""
    import numpy as np
    s = synth.config_mining(duration_s=args.duration_s)
    n, T = int(s["ids"].size), s["num_types"]
    iv = s["intervals"]
    ty = np.stack(np.meshgrid(np.arange(T), np.arange(T), np.arange(T), indexing="ij"),
                  -1).reshape(-1, 3)
    k = np.stack(np.meshgrid(np.arange(len(iv)), np.arange(len(iv)), indexing="ij"),
                 -1).reshape(-1, 2)
    M = ty.shape[0] * k.shape[0]
    lo_set = np.array([a for a, _ in iv], np.int32)
    hi_set = np.array([b for _, b in iv], np.int32)
    cand = {"types": np.repeat(ty, k.shape[0], 0).astype(np.int32),
            "len": np.full(M, 3, np.int32),
            "lo": np.tile(lo_set[k], (ty.shape[0], 1)).astype(np.int32),
            "hi": np.tile(hi_set[k], (ty.shape[0], 1)).astype(np.int32), "nmax": 3, "M": M}
    tick_s = 10_000
    cuts = np.searchsorted(s["ticks"], np.arange(1, int(np.ceil(args.duration_s /
                                                               args.partition_s)) + 1)
                           * args.partition_s * tick_s, side="left").tolist()
    cuts = sorted(set(min(c, n) for c in cuts) | {n})
    log("streaming: n=%d in %d partitions of %.0f s, M=%d" % (n, len(cuts), args.partition_s, M))
    ctx = fe.Context(0)
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    cd = ctx.cand_tensors(cand)
    cnt = torch.zeros(M, dtype=torch.int32, device=ctx.device)
    last = torch.full((M,), -1, dtype=torch.int32, device=ctx.device)

    def run_all():
        cnt.zero_()
        last.fill_(-1)
        prev, lat = 0, []
        for c in cuts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.count_resume(ids[:c], ticks[:c], T, cd, fe.FE_EXACT, prev, cnt, last)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            prev = c
        return lat
    run_all()
    lat = run_all()
    whole = ctx.count(ids, ticks, T, cd, fe.FE_EXACT)
    same = bool((whole == cnt).all())
    rec = []
    for j in range(0, len(cuts), 8):
        c = cuts[j]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.count(ids[:c], ticks[:c], T, cd, fe.FE_EXACT)
        torch.cuda.synchronize()
        rec.append((j, time.perf_counter() - t0))
    rec_total = sum(t for _, t in rec) * len(cuts) / len(rec)
    tot = sum(lat)
    ctx.close()
    return {"value": float("%.5g" % (M * n / tot)), "unit": "ee/s",
            "ms_per_partition": round(1e3 * tot / len(cuts), 3),
            "p50_ms": round(1e3 * float(np.median(lat)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "recount_estimate_s": round(rec_total, 3), "resume_total_s": round(tot, 4),
            "identical_to_whole_count": same,
            "config": {"workload": "streaming: mining recording in partitions, exact counts "
                                   "carried across partitions",
                       "n_events": n, "partitions": len(cuts), "partition_s": args.partition_s,
                       "candidates": M}}


CONTRACT_KEYS = ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling",
                 "vs_baseline", "dtype", "data")


def run_child(key, args):
    """One workload in a process of its own (so that workloads share no
    process state); returns its JSON object without the contract keys."""
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--workload", key,
           "--trace-s", str(args.trace_s), "--rate", str(args.rate),
           "--max-inflight", str(args.max_inflight)]
    t0 = time.perf_counter()
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=args.child_timeout_s)
    except subprocess.TimeoutExpired:
        log("%s: no result within %d s" % (key, args.child_timeout_s))
        return {"error": "timed out after %d s" % args.child_timeout_s}
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        log("%s: exit status %d" % (key, r.returncode))
        return {"error": "exit status %d" % r.returncode}
    d = json.loads(lines[-1])
    log("%s: %.1f s" % (key, time.perf_counter() - t0))
    return {k: v for k, v in d.items() if k not in CONTRACT_KEYS}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--duration-s", type=float, default=780.0,
                    help="stream duration of the mining workload (default 780 s)")
    ap.add_argument("--max-level", type=int, default=6)
    ap.add_argument("--cpu-baseline-s", type=float, default=8.0,
                    help="CPU oracle: seconds of work per timed run (3 runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="mining line only (no batched / served / large sub-objects)")
    ap.add_argument("--workload", default="mining",
                    choices=["mining", "batched", "served", "large", "streaming"],
                    help="mining (default, with the other workloads as sub-objects), or one "
                         "workload alone")
    ap.add_argument("--trace-s", type=float, default=12.0, help="served: trace length (s)")
    ap.add_argument("--rate", type=float, default=200.0, help="served: requests per second")
    ap.add_argument("--max-inflight", type=int, default=3,
                    help="served: rounds on the device at once (one stream each)")
    ap.add_argument("--partition-s", type=float, default=10.0,
                    help="streaming: seconds of recording per partition")
    ap.add_argument("--elimination", type=int, default=None, choices=[0, 1, 2],
                    help="mining: 1 = two passes at every level, 0 = one pass, 2 = the "
                         "library's per-level rule (default: the library's default)")
    ap.add_argument("--host-tiling", type=int, default=None, choices=[0, 1],
                    help="mining: 1 = tile each level on the host, 0 = on the device")
    ap.add_argument("--shared-lists", type=int, default=1, choices=[0, 1],
                    help="exact waves of join siblings keep lists 0..N-3 once (0 = per lane)")
    ap.add_argument("--type-dispatch", type=int, default=1, choices=[0, 1],
                    help="per-type dispatch for shared-prefix waves (0 = every event)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--child-timeout-s", type=int, default=300,
                    help="time limit of each sub-workload's process")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU: the counting path runs on a single device here; "
                  "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    extras = {}
    if args.workload == "mining" and not args.no_extras:
        # the other workloads first, each in a child process, before this
        # process uses the GPU
        for key in ("batched", "served", "large"):
            extras[key] = run_child(key, args)

    import torch
    from paper_0905_2200_amd import fe, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    fe.lib()  # fails loudly when the HIP library is not built
    common = {"n_gpus": 1, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
              "dtype": "int32", "data": "synthetic"}

    if args.workload != "mining":
        fn = {"batched": bench_batched, "served": bench_served, "large": bench_large,
              "streaming": bench_streaming}[args.workload]
        r = fn(args, fe, synth, torch)
        out = {"metric": "candidate-episode×events/s", "value": r.pop("value"),
               "unit": r.pop("unit", "ee/s"), "steps": args.steps, "warmup": args.warmup,
               **common, **r}
        print(json.dumps(out), flush=True)
        return

    m = bench_mining(args, fe, synth, torch)
    s = m.pop("stream")
    out = {"metric": "candidate-episode×events/s", "value": m["value"], "unit": "ee/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": m["ms_per_step"], "ms_per_mined_set": m["ms_per_step"],
           "p50_ms": m["p50_ms"], "p99_ms": m["p99_ms"],
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic", "config": m["config"],
           "roofline": m["roofline"], "stream_equivalent": m["stream_equivalent"],
           "dram": m["dram"]}
    out.update(extras)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_baseline_s)
        log("cpu baseline: %.1f s" % (time.perf_counter() - t0))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
