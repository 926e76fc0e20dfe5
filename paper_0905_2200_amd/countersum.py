"""Summarise rocprofv3 runs of the mining benchmark into profiles/.

    python -m paper_0905_2200_amd.countersum --trace DIR --fetch DIR --write DIR \
        --sq DIR [--sq DIR ...] --cmd-prefix "..." [--calib-mib 1024]

Each DIR is the output directory of one rocprofv3 run of
``bench.py --no-extras`` (a kernel trace with --stats, a FETCH_SIZE pass, a
WRITE_SIZE pass, and one or more passes of SQ counters).  Writes
profiles/map_counters.json -- per Map kernel (named as the library's kernel
timers name them, e.g. map_exact_n4_d2) the average per launch of every
counter, the calibrated beyond-L2 bytes and the average duration -- keyed by
a hash of the Map sources, which bench.py checks before it uses them; and
profiles/mining_counters.md, a readable summary with the commands.

FETCH_SIZE and WRITE_SIZE are scaled by what they read for one device copy
of --calib-mib MiB (bench.py --calib-copy-mib) in the same run.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
MAP_SOURCES = ["paper_0905_2200_amd/csrc/fe_map.h"] + [
    "paper_0905_2200_amd/csrc/fe_map_n%d.hip" % n for n in range(1, 9)]


def map_source_hash():
    h = hashlib.sha256()
    for p in MAP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def lib_name(kernel):
    """The library's timer name of a Map kernel (None for other kernels)."""
    m = re.search(r"k_map1?<(\d+), (true|false), (\d+), (true|false)>", kernel)
    if m:
        exact = m.group(2) == "true"
        return "map_%s_n%s_d%s" % ("exact" if exact else "relaxed", m.group(1),
                                   m.group(3) if exact else "1")
    m = re.search(r"k_deep<(\d+)>", kernel)
    if m:
        return "map_exact_n%s_deep" % m.group(1)
    return None


def _csv(d, suffix):
    f = glob.glob(os.path.join(d, "**", "*%s" % suffix), recursive=True)
    if not f:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return list(csv.DictReader(open(f[0])))


def counters(d):
    """{dispatch: (kernel, grid, {counter: value})} of a --pmc run."""
    out = {}
    for r in _csv(d, "counter_collection.csv"):
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        k = out.setdefault(key, [r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0), {}])
        name = r["Counter_Name"]
        k[2][name] = k[2].get(name, 0.0) + float(r["Counter_Value"])
    return out


def per_kernel(disp, names):
    """Average per launch of each counter in `names`, by library kernel name;
    and the same counters of the calibration copy."""
    acc = defaultdict(lambda: defaultdict(float))
    cnt = defaultdict(int)
    copy = None
    for kern, grid, vals in disp.values():
        # the calibration copy: the largest device copy of the run
        if "copyBuffer" in kern and vals and (copy is None or
                                              sum(vals.values()) > sum(copy.values())):
            copy = vals
        ln = lib_name(kern)
        if not ln:
            continue
        cnt[ln] += 1
        acc[ln]["grid"] += grid
        for n in names:
            acc[ln][n] += vals.get(n, 0.0)
    return {k: {n: v / cnt[k] for n, v in acc[k].items()} | {"launches": cnt[k]}
            for k in acc}, copy


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--sq", action="append", default=[])
    ap.add_argument("--calib-mib", type=int, default=1024)
    ap.add_argument("--cmd-prefix", default="rocprofv3")
    ap.add_argument("--bench-args", default="--steps 1 --warmup 1 --no-extras --no-cpu-baseline")
    a = ap.parse_args()

    # durations from the kernel trace
    dur = defaultdict(list)
    for r in _csv(a.trace, "kernel_trace.csv"):
        ln = lib_name(r["Kernel_Name"])
        if ln:
            dur[ln].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    fetch, cf = per_kernel(counters(a.fetch), ["FETCH_SIZE"])
    write, cw = per_kernel(counters(a.write), ["WRITE_SIZE"])
    sq = {}
    for d in a.sq:
        disp = counters(d)
        names = sorted({n for _, _, v in disp.values() for n in v})
        part, _ = per_kernel(disp, names)
        for k, v in part.items():
            sq.setdefault(k, {}).update(v)
    calib = a.calib_mib << 20
    ff = calib / (cf["FETCH_SIZE"] * 1024) if cf else 1.0
    wf = calib / (cw["WRITE_SIZE"] * 1024) if cw else 1.0
    kernels = {}
    for k in sorted(set(dur) | set(sq)):
        e = {"avg_ms": sum(dur[k]) / len(dur[k]) if dur.get(k) else None,
             "launches_traced": len(dur.get(k, []))}
        if k in fetch and k in write:
            e["fetch_kib"] = fetch[k]["FETCH_SIZE"]
            e["write_kib"] = write[k]["WRITE_SIZE"]
            e["hbm_bytes_per_launch"] = int(e["fetch_kib"] * 1024 * ff + e["write_kib"] * 1024 * wf)
        s = sq.get(k, {})
        for n, v in s.items():
            if n.startswith("SQ_"):
                e[n] = v
        if "SQ_INSTS_VALU" in s:
            e["valu_per_launch"] = s["SQ_INSTS_VALU"]
        if "SQ_INSTS_SALU" in s:
            e["salu_per_launch"] = s["SQ_INSTS_SALU"]
        if "grid" in s:
            e["waves"] = s["grid"] / 64
        kernels[k] = e
    out = {"map_source_hash": map_source_hash(),
           "calibration": {"copy_bytes": calib, "fetch_kib": cf and cf["FETCH_SIZE"],
                           "write_kib": cw and cw["WRITE_SIZE"], "fetch_factor": ff,
                           "write_factor": wf},
           "kernels": kernels}
    prof = os.path.join(ROOT, "profiles")
    json.dump(out, open(os.path.join(prof, "map_counters.json"), "w"), indent=1)

    # readable summary
    L = []
    L.append("# Map kernels of the mining workload: time, traffic and instruction issue\n")
    L.append("Workload: 64 neurons x 20 Hz x 780 s (1 057 255 events), levels 2-6, the "
             "library's default per-level elimination rule.  Commands (repo root, MI355X), one "
             "rocprofv3 run each:\n")
    L.append("```")
    base = "python3 bench.py %s --calib-copy-mib %d" % (a.bench_args, a.calib_mib)
    L.append("%s --kernel-trace --stats --output-format csv -d <dir> -o mining -- %s" % (
        a.cmd_prefix, base))
    L.append("%s --pmc FETCH_SIZE --output-format csv -d <dir> -o mining -- %s" % (
        a.cmd_prefix, base))
    L.append("%s --pmc WRITE_SIZE --output-format csv -d <dir> -o mining -- %s" % (
        a.cmd_prefix, base))
    L.append("%s --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
             "SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_INSTS_SMEM --output-format csv -d <dir> -o "
             "mining -- %s" % (a.cmd_prefix, base))
    L.append("python -m paper_0905_2200_amd.countersum --trace <dir> --fetch <dir> --write <dir> "
             "--sq <dir>")
    L.append("```\n")
    L.append("Calibration: a %d MiB device copy reads FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f "
             "KiB, so they are scaled by %.3f and %.3f.\n" % (
                 a.calib_mib, (cf or {}).get("FETCH_SIZE", 0), (cw or {}).get("WRITE_SIZE", 0),
                 ff, wf))
    L.append("Issue bound: a SIMD issues one wave64 VALU (or SALU) instruction every 4 cycles; "
             "256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G wave-instructions/s per kind.  "
             "`issue frac` = max(VALU, SALU) per launch / avg duration / 614.4e9.\n")
    L.append("| Kernel | launches | avg ms | waves | VALU/launch | SALU/launch | issue frac | "
             "LDS instr | LDS bank-conflict cycles / LDS instr | beyond-L2 bytes/launch | GB/s |")
    L.append("|---|---|---|---|---|---|---|---|---|---|---|")
    for k, e in sorted(kernels.items(), key=lambda kv: -(kv[1]["avg_ms"] or 0) *
                       kv[1]["launches_traced"]):
        if not e.get("avg_ms"):
            continue
        t = e["avg_ms"] * 1e-3
        iss = max(e.get("valu_per_launch", 0), e.get("salu_per_launch", 0))
        hb = e.get("hbm_bytes_per_launch")
        lds = e.get("SQ_INSTS_LDS")
        conf = e.get("SQ_LDS_BANK_CONFLICT")
        L.append("| %s | %d | %.3f | %s | %.3e | %.3e | %s | %s | %s | %s | %s |" % (
            k, e["launches_traced"], e["avg_ms"], "%.0f" % e["waves"] if "waves" in e else "-",
            e.get("valu_per_launch", 0), e.get("salu_per_launch", 0),
            "%.3f" % (iss / t / 614.4e9) if iss else "-",
            "%.3e" % lds if lds else "-",
            "%.2f" % (conf / lds) if lds and conf is not None else "-",
            "%.3e" % hb if hb else "-", "%.1f" % (hb / t / 1e9) if hb else "-"))
    L.append("\n`map_counters.json` holds these figures for `bench.py`, keyed by the hash %s of "
             "the Map sources they were taken on." % out["map_source_hash"])
    open(os.path.join(prof, "mining_counters.md"), "w").write("\n".join(L) + "\n")
    print(json.dumps({k: {kk: v[kk] for kk in ("avg_ms", "valu_per_launch", "salu_per_launch",
                                               "hbm_bytes_per_launch") if kk in v}
                      for k, v in kernels.items()}, indent=1))


if __name__ == "__main__":
    main()
