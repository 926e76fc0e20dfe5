#!/usr/bin/env python3
"""Throughput benchmark of the episode-counting hot path on one MI355X.

One step = one full level-wise mining run (Problem 1) on the mining
workload: 64 neurons firing at 20 Hz for 780 s (about 1.05M events, int32
ids and 0.1 ms int32 ticks) with eight planted cascades of 3-6 nodes, hop
intervals {(0,5], (5,10], (10,20]} ms, levels 2-6, threshold 0.5 Hz x 780 s
= 390.  Every level is generated on the host and counted on the GPU with
two-pass elimination (relaxed pass, elimination, exact pass on survivors),
each pass by MapConcatenate Map/Concatenate kernels.

Metric: candidate-episode x events per second, where a step's work is
sum over levels >= 2 of (candidates + survivors) x n events.  The stream
is resident in HBM before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_EE = 8  # one int32 id + one int32 tick per event per candidate machine
MAP_SOURCES = ["paper_0905_2200_amd/csrc/fe_map.h"] + [
    "paper_0905_2200_amd/csrc/fe_map_n%d.hip" % n for n in range(1, 9)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def map_source_hash():
    h = hashlib.sha256()
    for p in MAP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current Map sources (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("map_source_hash") != map_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(stream, target_s, n_types, intervals, theta):
    """The oracle's two-pass counter (projection mode, all host threads) on
    a seeded uniform sample of the level-3 candidate set of the same
    workload (random 3-node episodes over the 64 types and the interval
    set), grown until about target_s seconds of CPU work."""
    import numpy as np
    import oracle
    from paper_0905_2200_amd import synth
    ids, ticks = stream["ids"], stream["ticks"]
    rng = np.random.default_rng([2, 777])
    total_ee, total_s, M_done = 0.0, 0.0, 0
    chunk = 2000
    threads = oracle.max_threads()
    while total_s < target_s and M_done < 2_000_000:
        eps = synth.random_episodes(rng, chunk, n_types, 3, intervals)
        c = synth.pack(eps)
        t0 = time.perf_counter()
        up, ex = oracle.two_pass(ids, ticks, n_types, c["types"], c["len"], c["lo"], c["hi"],
                                 theta, projection=True, nthreads=threads)
        dt = time.perf_counter() - t0
        total_s += dt
        total_ee += float(chunk + int((up >= theta).sum())) * ids.size
        M_done += chunk
        if dt < target_s / 8:
            chunk *= 2
    # single thread, plain configuration (all 4096 pairs over about 2e4 events)
    pl = synth.config_plain()
    pc = pl["candidates"]
    reps, t0 = 0, time.perf_counter()
    while reps == 0 or time.perf_counter() - t0 < 1.0:
        up1, _ = oracle.two_pass(pl["ids"], pl["ticks"], 64, pc["types"], pc["len"], pc["lo"],
                                 pc["hi"], pl["theta"], projection=True, nthreads=1)
        reps += 1
    dt1 = time.perf_counter() - t0
    ee1 = reps * float(pc["M"] + int((up1 >= pl["theta"]).sum())) * pl["ids"].size
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": total_ee / total_s, "unit": "ee/s", "cores": threads, "kind": "oracle",
            "sample": ("two-pass (relaxed pass, elimination, exact pass) in projection mode on "
                       "%d random level-3 episodes of the mining workload over its %d events, "
                       "%.1f s" % (M_done, ids.size, total_s)),
            "cpu_model": model,
            "single_thread_plain": {"value": float("%.4g" % (ee1 / dt1)),
                                    "unit": "ee/s",
                                    "sample": "two-pass over the 4096 pairs of the plain "
                                              "configuration (%d events), 1 thread, %d runs "
                                              "in %.2f s" % (pl["ids"].size, reps, dt1)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--duration-s", type=float, default=780.0,
                    help="stream duration of the mining workload (default 780 s)")
    ap.add_argument("--max-level", type=int, default=6)
    ap.add_argument("--cpu-baseline-s", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="mining",
                    choices=["mining", "batched", "served", "streaming"],
                    help="mining (default): level-wise mining of one stream; batched: 64 "
                         "recordings, one planned batch vs per-recording launches; served: "
                         "window requests from 32 arrays, open-loop Poisson trace")
    ap.add_argument("--trace-s", type=float, default=20.0, help="served: trace length (s)")
    ap.add_argument("--rate", type=float, default=200.0, help="served: requests per second")
    ap.add_argument("--max-inflight", type=int, default=3,
                    help="served: rounds on the device at once (one stream each)")
    ap.add_argument("--partition-s", type=float, default=10.0,
                    help="streaming: seconds of recording per partition")
    ap.add_argument("--one-pass", action="store_true",
                    help="mining: Algorithm 1 over every candidate, no elimination pass")
    ap.add_argument("--host-tiling", type=int, default=None, choices=[0, 1],
                    help="mining: 1 = tile each level on the host, 0 = on the device "
                         "(default: the library's)")
    ap.add_argument("--type-dispatch", type=int, default=1, choices=[0, 1],
                    help="per-type dispatch for shared-prefix waves (0 = every event)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU: the counting path runs on a single device here; "
                  "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_0905_2200_amd import fe, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    fe.lib()  # fails loudly when the HIP library is not built
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "streaming":
        return bench_streaming(args)

    s = synth.config_mining(duration_s=args.duration_s)
    n = int(s["ids"].size)
    theta, intervals = s["theta"], s["intervals"]
    log("workload: %s; n=%d theta=%d" % (s["name"], n, theta))

    ctx = fe.Context(0)
    ctx.set_param(fe.PARAM_TYPE_DISPATCH, args.type_dispatch)
    ctx.set_param(fe.PARAM_ELIMINATION, 0 if args.one_pass else 1)
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
        log("warmup step %d: %.2f s" % (w, time.perf_counter() - t0))

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

    ee_step = sum((lv["n_candidates"] + (0 if args.one_pass else lv["n_survivors"])) * n
                  for lv in res if lv["level"] >= 2)
    value = ee_step * args.steps / t_total
    for lv in res:
        log("level %d: candidates %d survivors %d frequent %d gen %.1f ms count %.1f ms" % (
            lv["level"], lv["n_candidates"], lv["n_survivors"], lv["n_frequent"],
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
    roofline = None
    if dom:
        name, v = dom
        achieved = BYTES_PER_EE * v["ee"] / (v["total_ms"] * 1e-3) / 1e9
        tb = traffic_for(name)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": tb, "kernel": name,
                    "avg_launch_ms": round(v["total_ms"] / v["launches"], 4),
                    "launches": v["launches"],
                    "ee_per_s": v["ee"] / (v["total_ms"] * 1e-3)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(s, args.cpu_baseline_s, s["num_types"], intervals, theta)
        cpu["value"] = float("%.4g" % cpu["value"])

    times_ms = sorted(1e3 * t for t in times)
    out = {
        "metric": "candidate-episode×events/s",
        "value": float("%.5g" % value),
        "unit": "ee/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_total / args.steps, 2),
        "p50_ms": round(float(np.percentile(times_ms, 50)), 2),
        "p99_ms": round(float(np.percentile(times_ms, 99)), 2),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "level-wise mining, %s, levels 2-%d" % (
                       "one pass (no elimination)" if args.one_pass else "two-pass",
                       args.max_level),
                   "neurons": s["num_types"], "rate_hz": 20, "duration_s": args.duration_s,
                   "n_events": n, "theta": theta, "intervals_ticks": intervals,
                   "ee_per_step": ee_step,
                   "levels": [{k: lv[k] for k in ("level", "n_candidates", "n_survivors",
                                                   "n_frequent")} for lv in res]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_batched(args):
    """64 recordings of uneven length (1e4-1e6 events), 16-256 neurons, each
    with its own 1e3-5e4 candidates of 2-8 nodes; one step = the two-pass
    count of every recording.  Batched: one planned batch (persistent
    launches, one captured graph per episode size, autotuned launch shape).
    Plain: one fe_count_two_pass call per recording."""
    import numpy as np
    import torch
    from paper_0905_2200_amd import fe, synth
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
        outs = []
        for d in dev:
            outs.append(ctx.count_two_pass(d["ids"], d["ticks"], d["num_types"], d["cand"],
                                           d["theta"]))
        torch.cuda.synchronize()
        return outs

    for _ in range(max(args.warmup, 1)):
        outs = plain()
    tp = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        outs = plain()
        tp.append(time.perf_counter() - t0)
    log("plain: %s s" % ["%.3f" % t for t in tp])

    t0 = time.perf_counter()
    b = fe.Batch(ctx, dev)
    t_plan = time.perf_counter() - t0
    tun = b.autotune(reps=2)
    log("batch plan %.2f s; autotuned %s" % (t_plan, tun))
    for _ in range(max(args.warmup, 1)):
        b.run()
    torch.cuda.synchronize()
    tb = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    log("batched: %s s" % ["%.4f" % t for t in tb])
    same = all(bool((b.upper[r] == o[0]).all()) and bool((b.exact[r] == o[1]).all())
               for r, o in enumerate(outs))
    ee = 0
    for r, d in enumerate(dev):
        ns = int((b.upper[r] >= d["theta"]).sum())
        ee += (d["cand"]["M"] + ns) * d["ids"].numel()
    tbm, tpm = float(np.median(tb)), float(np.median(tp))
    out = {"metric": "candidate-episode×events/s", "value": float("%.5g" % (ee / tbm)),
           "unit": "ee/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * tbm, 3), "p50_ms": round(1e3 * tbm, 3),
           "p99_ms": round(1e3 * float(np.percentile(tb, 99)), 3),
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": "batched: 64 recordings, two-pass counting",
                      "recordings": len(recs), "events": int(sum(r["ids"].size for r in recs)),
                      "candidates": int(sum(r["candidates"]["M"] for r in recs)),
                      "ee_per_step": ee, "tuning": tun},
           "plain": {"value": float("%.5g" % (ee / tpm)), "ms_per_step": round(1e3 * tpm, 2)},
           "batched_over_plain": round(tpm / tbm, 2), "identical_results": same}
    print(json.dumps(out), flush=True)
    b.close()
    ctx.close()


def bench_streaming(args):
    """The mining recording arriving in partitions of --partition-s seconds,
    with every 3-node episode over its 64 neurons x the interval set resident
    (2.36 M candidates, the level-3 candidate set); after each partition the
    exact counts over the recording so far are brought up to date by
    fe_count_resume (carried count and last completion per candidate).
    Compared with recounting the whole prefix with fe_count."""
    import numpy as np
    import torch
    from paper_0905_2200_amd import fe, synth
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
    tick_s = 10_000  # ticks per second (0.1 ms)
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

    run_all()  # warm-up
    lat = run_all()
    whole = ctx.count(ids, ticks, T, cd, fe.FE_EXACT)
    same = bool((whole == cnt).all())
    # recounting each prefix instead (every 8th partition, scaled to all)
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
    ee = M * n
    out = {"metric": "candidate-episode×events/s", "value": float("%.5g" % (ee / tot)),
           "unit": "ee/s", "n_gpus": 1, "steps": len(cuts), "warmup": 1,
           "ms_per_step": round(1e3 * tot / len(cuts), 3),
           "p50_ms": round(1e3 * float(np.median(lat)), 3),
           "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": "streaming: mining recording in partitions, exact counts "
                                  "carried across partitions",
                      "n_events": n, "partitions": len(cuts), "partition_s": args.partition_s,
                      "candidates": M},
           "recount_estimate_s": round(rec_total, 3),
           "resume_total_s": round(tot, 4), "identical_to_whole_count": same}
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_served(args):
    """32 simulated arrays (64-256 neurons, 20 Hz) stream events; window
    requests (1-60 s) arrive as a Poisson process; each is the two-pass count
    of 50 000 resident episodes (2-6 nodes) over the window.  Served: the
    library's continuous-batching server.  Plain: the same trace handled
    first-in first-out, one fe_count_two_pass call per request.  Latency =
    completion - scheduled arrival."""
    import numpy as np
    import torch
    from paper_0905_2200_amd import fe, synth
    t0 = time.perf_counter()
    sv = synth.config_served(trace_s=args.trace_s, rate_req=args.rate)
    reqs = sv["requests"]
    arrays = sv["arrays"]
    log("served workload: %d arrays, %d events, %d requests over %.0f s, M=%d (%.1f s to generate)"
        % (len(arrays), sum(a["ids"].size for a in arrays), len(reqs), args.trace_s,
           sv["candidates"]["M"], time.perf_counter() - t0))
    ctx = fe.Context(0)
    tick_ns = 100_000  # 0.1 ms

    def window(a, t0_, t1_):
        ar = arrays[a]
        return (int(np.searchsorted(ar["ticks"], t0_, "left")),
                int(np.searchsorted(ar["ticks"], t1_, "left")))

    spans = [window(r["array"], r["t_begin"], r["t_end"]) for r in reqs]
    preroll_ticks = int(sv["preroll_s"] * 10000)

    # ---------------------------------------------------------------- served
    server = fe.Server(ctx, sv["candidates"], [a["num_types"] for a in arrays],
                       capacity=max(a["ids"].size for a in arrays) + 16,
                       hbm_budget=16 << 30, max_inflight=args.max_inflight, max_round=64)
    ptr = [0] * len(arrays)

    def feed(upto):  # append every array's events with tick < upto
        for k, a in enumerate(arrays):
            e = int(np.searchsorted(a["ticks"], upto, "left"))
            if e > ptr[k]:
                server.append(k, a["ids"][ptr[k]:e], a["ticks"][ptr[k]:e])
                ptr[k] = e

    feed(preroll_ticks)
    # warm-up: a few requests before the clock starts
    for r in reqs[:8]:
        server.wait(server.submit(r["array"], r["t_begin"], min(r["t_end"], preroll_ticks),
                                  r["theta"]))
    base = time.monotonic_ns() + 200_000_000
    tickets = []
    done = {}
    for k, r in enumerate(reqs):
        due = base + int(r["arrival_s"] * 1e9)
        feed(preroll_ticks + int(r["arrival_s"] * 10000) + 1)
        while time.monotonic_ns() < due:
            pass
        tickets.append(server.submit(r["array"], r["t_begin"], r["t_end"], r["theta"], due))
    for k, t in enumerate(tickets):
        done[k] = server.wait(t, copy=(k % 50 == 0))
    stats = server.stats()
    lat = np.array([(done[k]["done_ns"] - done[k]["arrival_ns"]) / 1e6 for k in range(len(reqs))])
    wall = (max(d["done_ns"] for d in done.values()) - base) / 1e9
    ee = sum((sv["candidates"]["M"] + done[k]["n_survivors"]) * done[k]["n_events"]
             for k in range(len(reqs)))
    rounds = [done[k]["round_size"] for k in range(len(reqs))]
    log("served: p50 %.1f ms p99 %.1f ms, wall %.2f s, stats %s, mean round %.1f" % (
        np.percentile(lat, 50), np.percentile(lat, 99), wall, stats, np.mean(rounds)))

    # ---------------------------------------------------------------- plain FIFO
    dev = [ctx.stream_tensors(a["ids"], a["ticks"]) for a in arrays]
    dc = ctx.cand_tensors(sv["candidates"])
    torch.cuda.synchronize()
    same = True
    plat = []
    cap_s = 3.0 * args.trace_s + 10
    base = time.monotonic_ns() + 200_000_000
    for k, r in enumerate(reqs):
        due = base + int(r["arrival_s"] * 1e9)
        while time.monotonic_ns() < due:
            pass
        a, b = spans[k]
        ids, ticks = dev[r["array"]]
        up, ex, ns = ctx.count_two_pass(ids[a:b], ticks[a:b], arrays[r["array"]]["num_types"], dc,
                                        r["theta"])
        torch.cuda.synchronize()
        plat.append((time.monotonic_ns() - due) / 1e6)
        if "upper" in done[k]:
            same &= bool((up.cpu().numpy() == done[k]["upper"]).all()
                         and (ex.cpu().numpy() == done[k]["exact"]).all())
        if (time.monotonic_ns() - base) / 1e9 > cap_s:
            log("plain: stopped after %d of %d requests (%.0f s cap)" % (k + 1, len(reqs), cap_s))
            break
    plat = np.array(plat)
    log("plain: p50 %.1f ms p99 %.1f ms over %d requests" % (
        np.percentile(plat, 50), np.percentile(plat, 99), plat.size))
    out = {"metric": "candidate-episode×events/s", "value": float("%.5g" % (ee / wall)),
           "unit": "ee/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": round(1e3 * wall, 1), "p50_ms": round(float(np.percentile(lat, 50)), 2),
           "p99_ms": round(float(np.percentile(lat, 99)), 2), "higher_is_better": True,
           "scaling": "strong", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "served: 32 arrays, Poisson window requests",
                      "requests": len(reqs), "rate_per_s": args.rate, "trace_s": args.trace_s,
                      "resident_episodes": sv["candidates"]["M"], "ee_total": ee,
                      "rounds": stats["rounds"], "mean_round_size": round(float(np.mean(rounds)), 2),
                      "max_inflight_seen": stats["max_inflight_seen"]},
           "plain_fifo": {"p50_ms": round(float(np.percentile(plat, 50)), 2),
                          "p99_ms": round(float(np.percentile(plat, 99)), 2),
                          "requests_done": int(plat.size)},
           "identical_results": same}
    print(json.dumps(out), flush=True)
    server.close()
    ctx.close()


if __name__ == "__main__":
    main()
