"""Write the oracle's expected outputs for the full-size workloads.

    python -m tests.golden.make_fullsize {mining,large,batched,served} [--threads K]

Calls only the seeded input generators (paper_0905_2200_amd.synth, which
hold none of the counting arithmetic) and the CPU oracle (oracle/).  The GPU
tests (tests/test_gpu_fullsize.py) regenerate the same inputs, check their
fingerprint against the one stored here, and compare the library's outputs
with these values element by element.  Each file takes minutes to an hour of
CPU time to write, which is why the values are stored rather than recomputed
on every GPU run.

What each file holds (int32 counts; "exact for every candidate" means the
Algorithm 1 count also of candidates the relaxed pass prunes, so that either
form of the library's output -- two-pass with -1 for pruned candidates, or
one pass -- can be checked):

* fullsize_mining.npz -- the mining workload (64 neurons x 20 Hz x 780 s,
  levels 2-6, threshold 390): per level the number of candidates and of
  pass-1 survivors, and the whole frequent set with relaxed and exact counts;
  every candidate of levels 2, 5 and 6 with both counts; for levels 3 and 4
  a stated seeded sample with both counts: the 16384 candidates of the 256
  consecutive 64-candidate tiles starting at a seeded tile of the generation
  order (every survivor among them included), 20000 seeded random
  candidates, and every planted sub-episode of the level.
* fullsize_large.npz -- the large-array workload (256 neurons, about 1.1e7
  events): both 1e5-candidate sets (N = 3 and N = 4), both counts of every
  candidate.
* fullsize_batched.npz -- the batched workload (64 recordings, 727774
  candidates of 2-8 nodes): both counts of every candidate of every recording.
* fullsize_served.npz -- the served workload's full 60 s trace (about 12000
  window requests over 32 arrays, 50000 resident episodes): for a seeded
  sample of 5% of the requests (at least 600), the window's event count, the
  numbers of survivors and frequent episodes, and SHA-256 digests of the
  request's whole upper and two-pass exact arrays (int32 little endian).
"""
from __future__ import annotations

import argparse
import hashlib
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import mine  # noqa: E402
from paper_0905_2200_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE_TILES = 256      # consecutive 64-candidate tiles in the mining sample
SAMPLE_RANDOM = 20000   # random candidates in the mining sample
SERVED_FRACTION = 0.05


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(np.asarray(a), dtype="<i4").tobytes())
    return h.hexdigest()


def stream_fingerprint(ids, ticks, *extra):
    return digest(ids, ticks, *[np.asarray(e) for e in extra])


def cand_fingerprint(c):
    return digest(c["types"], c["len"], c["lo"], c["hi"])


def both_counts(ids, ticks, T, c, threads):
    up = oracle.count(ids, ticks, T, c["types"], c["len"], c["lo"], c["hi"], oracle.MODE_RELAXED,
                      projection=True, nthreads=threads)
    ex = oracle.count(ids, ticks, T, c["types"], c["len"], c["lo"], c["hi"], oracle.MODE_EXACT,
                      projection=True, nthreads=threads)
    return up.astype(np.int32), ex.astype(np.int32)


def rows_of(types, lo, hi):
    return np.concatenate([types, lo, hi], axis=1).astype(np.int64)


def find_rows(rows, want):
    """Indices into rows of each row of want (-1 when absent)."""
    if want.shape[0] == 0:
        return np.zeros(0, np.int64)
    v = np.dtype((np.void, 8 * rows.shape[1]))
    rv = np.ascontiguousarray(rows).view(v).ravel()
    wv = np.ascontiguousarray(want).view(v).ravel()
    order = np.argsort(rv, kind="stable")
    pos = np.searchsorted(rv[order], wv)
    pos = np.minimum(pos, rv.size - 1)
    return np.where(rv[order][pos] == wv, order[pos], -1)


def make_mining(threads):
    s = synth.config_mining()
    ids, ticks, T, theta = s["ids"], s["ticks"], s["num_types"], s["theta"]
    out = {"fingerprint": stream_fingerprint(ids, ticks, np.asarray(s["intervals"]), [theta]),
           "theta": theta, "max_level": 6}
    rng = np.random.default_rng(20260)

    def pick(level, M):
        if level in (2, 5, 6):
            return True
        if level not in (3, 4):
            return None
        tiles = M // 64
        t0 = int(rng.integers(0, max(tiles - SAMPLE_TILES, 1)))
        block = np.arange(t0 * 64, min(M, (t0 + SAMPLE_TILES) * 64))
        rnd = rng.choice(M, min(SAMPLE_RANDOM, M), replace=False)
        out["sample_block_%d" % level] = np.array([t0 * 64, block.size])
        return np.union1d(block, rnd)

    def planted(level):
        eps = [e for c in s["cascades"] for e in synth.sub_episodes(c, level)]
        if not eps:
            return np.zeros((0, 3 * level - 2), np.int64)
        p = synth.pack(eps, nmax=level)
        return rows_of(p["types"], p["lo"], p["hi"])

    def on_level(level, info):
        L = level
        out["n_candidates_%d" % L] = info["n_candidates"]
        out["n_survivors_%d" % L] = info["n_survivors"]
        for k in ("types", "lo", "hi", "upper", "exact"):
            out["F_%s_%d" % (k, L)] = np.asarray(info[k]).astype(np.int32)
        if "all_types" in info:
            for k in ("types", "lo", "hi", "upper", "exact"):
                out["all_%s_%d" % (k, L)] = np.asarray(info["all_" + k]).astype(np.int32)
        if "sample_idx" in info:
            for k in ("idx", "types", "lo", "hi", "upper", "exact"):
                out["s_%s_%d" % (k, L)] = np.asarray(info["sample_" + k]).astype(np.int32)
        print("level %d: %d candidates, %d survivors, %d frequent (%.0f s)" % (
            L, info["n_candidates"], info["n_survivors"], info["types"].shape[0],
            time.time() - t_start), flush=True)
        # checkpoint: the levels done so far ("complete" is set at the end)
        done.append(L)
        save(False)

    def save(complete):
        out["levels_done"] = np.array([1] + done, np.int32)
        out["complete"] = complete
        tmp = os.path.join(HERE, "fullsize_mining.tmp.npz")
        np.savez_compressed(tmp, **out)
        os.replace(tmp, os.path.join(HERE, "fullsize_mining.npz"))

    hist = np.bincount(ids, minlength=T)
    F1 = np.nonzero(hist >= theta)[0]
    out["n_candidates_1"] = T
    out["n_survivors_1"] = T
    out["F_types_1"] = F1[:, None].astype(np.int32)
    out["F_lo_1"] = np.zeros((F1.size, 0), np.int32)
    out["F_hi_1"] = np.zeros((F1.size, 0), np.int32)
    out["F_upper_1"] = hist[F1].astype(np.int32)
    out["F_exact_1"] = hist[F1].astype(np.int32)
    done = []
    t_start = time.time()
    res = mine.mine_arrays(ids, ticks, T, s["intervals"], theta, 6, nthreads=threads,
                           keep=pick, planted=planted, on_level=on_level)
    out["n_candidates_1"] = T
    out["n_survivors_1"] = T
    for k in ("types", "lo", "hi", "upper", "exact"):
        out["F_%s_1" % k] = np.asarray(res[1][k]).astype(np.int32)
    out["levels"] = np.array(sorted(res), np.int32)
    save(True)


def make_large(threads):
    s = synth.config_large()
    out = {"fingerprint": stream_fingerprint(s["ids"], s["ticks"], [s["theta"]]),
           "theta": s["theta"]}
    for N, c in s["candidate_sets"].items():
        t0 = time.time()
        up, ex = both_counts(s["ids"], s["ticks"], s["num_types"], c, threads)
        out["cand_fp_%d" % N] = cand_fingerprint(c)
        out["upper_%d" % N] = up
        out["exact_%d" % N] = ex
        print("large N=%d: %d candidates, %d survivors (%.0f s)" % (
            N, c["M"], int((up >= s["theta"]).sum()), time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "fullsize_large.npz"), **out)


def make_batched(threads):
    recs = synth.config_batched()
    ups, exs, off, fps = [], [], [0], []
    t0 = time.time()
    for r in recs:
        c = r["candidates"]
        up, ex = both_counts(r["ids"], r["ticks"], r["num_types"], c, threads)
        ups.append(up)
        exs.append(ex)
        off.append(off[-1] + c["M"])
        fps.append(stream_fingerprint(r["ids"], r["ticks"], [r["theta"]]) + cand_fingerprint(c))
    out = {"fingerprint": digest(np.frombuffer("".join(fps).encode(), np.uint8)),
           "upper": np.concatenate(ups), "exact": np.concatenate(exs),
           "offsets": np.array(off, np.int64), "theta": np.array([r["theta"] for r in recs])}
    print("batched: %d recordings, %d candidates (%.0f s)" % (len(recs), off[-1],
                                                              time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "fullsize_batched.npz"), **out)


def make_served(threads):
    sv = synth.config_served(trace_s=60.0)
    reqs, arrays, c = sv["requests"], sv["arrays"], sv["candidates"]
    k = min(len(reqs), max(600, int(math.ceil(SERVED_FRACTION * len(reqs)))))
    rng = np.random.default_rng(5005)
    idx = np.sort(rng.choice(len(reqs), k, replace=False))
    fields = {"n_events": [], "n_survivors": [], "n_frequent": [], "upper_sha": [],
              "exact_sha": []}
    t0 = time.time()
    for j, i in enumerate(idx):
        r = reqs[i]
        a = arrays[r["array"]]
        b, e = (int(np.searchsorted(a["ticks"], r["t_begin"], "left")),
                int(np.searchsorted(a["ticks"], r["t_end"], "left")))
        up, ex = oracle.two_pass(a["ids"][b:e], a["ticks"][b:e], a["num_types"], c["types"],
                                 c["len"], c["lo"], c["hi"], r["theta"], projection=True,
                                 nthreads=threads)
        fields["n_events"].append(e - b)
        fields["n_survivors"].append(int((up >= r["theta"]).sum()))
        fields["n_frequent"].append(int((ex >= r["theta"]).sum()))
        fields["upper_sha"].append(digest(up))
        fields["exact_sha"].append(digest(ex))
        if j % 100 == 0:
            print("served: %d of %d sampled requests (%.0f s)" % (j, k, time.time() - t0),
                  flush=True)
    fp = digest(np.array([[r["array"], r["t_begin"], r["t_end"], r["theta"]] for r in reqs]),
                *[np.concatenate([a["ids"], a["ticks"]]) for a in arrays],
                c["types"], c["len"], c["lo"], c["hi"])
    out = {"fingerprint": fp, "sample": idx, "n_requests": len(reqs)}
    for kk, v in fields.items():
        out[kk] = np.array(v)
    np.savez_compressed(os.path.join(HERE, "fullsize_served.npz"), **out)
    print("served: %d of %d requests (%.0f s)" % (k, len(reqs), time.time() - t0), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("which", nargs="+", choices=["mining", "large", "batched", "served"])
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for w in a.which:
        {"mining": make_mining, "large": make_large, "batched": make_batched,
         "served": make_served}[w](a.threads)


if __name__ == "__main__":
    main()
