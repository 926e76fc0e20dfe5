"""Measure where the whole-stream Map (the paper's PTPE, P = 1) overtakes
MapConcatenate (P > 1 segments) on this GPU, per episode size N, and fit the
crossover tile count C(N) = a/N + b (the hybrid rule of Algorithm 2 with the
size penalty f(N) of Eq. 2; the paper's Table 1 and its a/N + b fit, Sec. 6.2).

    python -m paper_0905_2200_amd.crossover [--quick]

prints one JSON line: the measured table and the fitted (a, b) for the
exact and relaxed counters.  The library's defaults for
FE_PARAM_CROSSOVER_A / _B come from this measurement on an MI355X.
Candidates are tiles of join siblings (shared first N-1 types and first
N-2 hops) over the mining recording, as level-wise mining produces them."""
import argparse
import json
import sys
import time

import numpy as np


def sibling_tiles(rng, tiles, N, num_types, intervals):
    """tiles x 64 candidates; each tile shares its first N-1 types and its
    first N-2 hops (the join siblings of one episode), each lane draws its
    last type and last hop."""
    M = tiles * 64
    pre = rng.integers(0, num_types, size=(tiles, max(N - 1, 1)))
    types = np.empty((M, N), np.int32)
    types[:, :N - 1] = np.repeat(pre[:, :N - 1], 64, axis=0)
    types[:, N - 1] = rng.integers(0, num_types, size=M)
    k = rng.integers(0, len(intervals), size=(M, max(N - 1, 1)))[:, :N - 1]
    if N >= 3:
        kt = rng.integers(0, len(intervals), size=(tiles, N - 2))
        k[:, :N - 2] = np.repeat(kt, 64, axis=0)
    lo = np.array([a for a, _ in intervals], np.int32)[k]
    hi = np.array([b for _, b in intervals], np.int32)[k]
    return {"types": types, "len": np.full(M, N, np.int32), "lo": np.ascontiguousarray(lo),
            "hi": np.ascontiguousarray(hi), "nmax": N, "M": M}


def timed(ctx, torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def crossover_tiles(tiles, ratio):
    """Tile count from which on P = 1 stays at least as fast (ratio = t(P=1)
    / t(best P>1) <= 1 at it and every larger size), interpolated in
    log2(tiles) after the last size where segmenting wins; None if never."""
    last = max((j for j, r in enumerate(ratio) if r > 1.0), default=-1)
    if last == len(ratio) - 1:
        return None
    if last < 0:
        return float(tiles[0])
    x0, x1 = np.log2(tiles[last]), np.log2(tiles[last + 1])
    r0, r1 = np.log(ratio[last]), np.log(ratio[last + 1])
    x = x0 + (x1 - x0) * (r0 / (r0 - r1)) if r0 != r1 else x1
    return float(2.0 ** x)


def fit_a_over_n_plus_b(Ns, C):
    A = np.stack([1.0 / np.asarray(Ns, float), np.ones(len(Ns))], 1)
    (a, b), *_ = np.linalg.lstsq(A, np.asarray(C, float), rcond=None)
    return float(a), float(b)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer sizes (a smoke run)")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    import torch
    from paper_0905_2200_amd import fe, synth
    s = synth.config_mining()
    ctx = fe.Context(0)
    ids, ticks = ctx.stream_tensors(s["ids"], s["ticks"])
    rng = np.random.default_rng(99)
    Ns = [2, 3, 4] if args.quick else [2, 3, 4, 5, 6, 7, 8]
    tiles = [256, 1024, 4096] if args.quick else [512, 1024, 2048, 4096, 8192, 16384, 32768]
    target = ctx.get_param(fe.PARAM_TARGET_WAVES)  # the automatic P's aim
    out = {"n_events": int(s["ids"].size), "tiles": tiles, "target_waves": target,
           "table": {}, "fit": {}}
    for mode, name in ((fe.FE_EXACT, "exact"), (fe.FE_RELAXED, "relaxed")):
        cross = []
        for N in Ns:
            ratios = []
            for t in tiles:
                cand = ctx.cand_tensors(sibling_tiles(rng, t, N, s["num_types"], s["intervals"]))

                def run(P):
                    ctx.set_param(fe.PARAM_SEGMENTS, P)
                    return timed(ctx, torch, lambda: ctx.count(ids, ticks, s["num_types"], cand,
                                                               mode), args.reps)
                t1 = run(1)
                base = max(2, -(-target // t))
                tp = min(run(P) for P in sorted({max(2, base // 2), base, 2 * base}))
                ratios.append(t1 / tp)
                print("%s N=%d tiles=%d: P=1 %.2f ms, best P>1 %.2f ms" % (
                    name, N, t, 1e3 * t1, 1e3 * tp), file=sys.stderr, flush=True)
            ctx.set_param(fe.PARAM_SEGMENTS, 0)
            c = crossover_tiles(tiles, ratios)
            out["table"]["%s_n%d" % (name, N)] = {"ratio_p1_over_best": [round(r, 3) for r in ratios],
                                                   "crossover_tiles": c}
            if c is not None:
                cross.append((N, c))
        if len(cross) >= 2:
            a, b = fit_a_over_n_plus_b([n for n, _ in cross], [c for _, c in cross])
            out["fit"][name] = {"a": round(a, 1), "b": round(b, 1), "points": cross}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
