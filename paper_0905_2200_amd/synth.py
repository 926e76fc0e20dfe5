"""Seeded synthetic spike streams and candidate sets.

This module only draws random numbers and arranges them; it holds none of the
counting arithmetic.  Both the GPU tests/benchmark and the CPU oracle take
their inputs from here.

The streams copy the shape of the paper's data (Sec. 6.1): multi-electrode
array spike trains, one event type per neuron, Poisson background firing plus
embedded causal chains ("cascades") whose hops have delays inside an
interval.  Timestamps are int32 ticks of 0.1 ms; a delay interval (a, b] in
milliseconds is (10a, 10b] in ticks.  Events are ordered by (tick, id).

Generator rules:
* background: for every neuron, count ~ Poisson(rate * T), times uniform over
  [0, T), floored to ticks;
* cascades: distinct neurons; each hop has an interval from the interval set
  and each firing draws its delay uniformly from the integer ticks of that
  interval; onsets are a Poisson process at the cascade's rate, thinned so
  that two onsets of one cascade are more than the cascade's span apart;
* every generator is seeded with ``numpy.random.default_rng([tag, run])``.
"""
from __future__ import annotations

import math

import numpy as np

TICKS_PER_MS = 10
# (0,5], (5,10], (10,20] ms in 0.1 ms ticks
INTERVALS = [(0, 50), (50, 100), (100, 200)]


def rng_for(tag: int, run: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(tag), int(run)])


def sort_events(ids, ticks):
    ids = np.asarray(ids, np.int64)
    ticks = np.asarray(ticks, np.int64)
    order = np.lexsort((ids, ticks))
    return ids[order].astype(np.int32), ticks[order].astype(np.int32)


def background(rng, rates_hz, duration_ticks):
    """Homogeneous Poisson firing per neuron (one event type per neuron)."""
    rates_hz = np.asarray(rates_hz, np.float64)
    T_s = duration_ticks / (1000.0 * TICKS_PER_MS)
    counts = rng.poisson(rates_hz * T_s)
    ids = np.repeat(np.arange(len(rates_hz), dtype=np.int64), counts)
    ticks = np.floor(rng.random(ids.size) * duration_ticks).astype(np.int64)
    return ids, ticks


def cascade_firings(rng, neurons, intervals, duration_ticks, rate_hz=None,
                    n_firings=None):
    """Plant one cascade.  Returns (ids, ticks, onsets) of its events.

    Either ``rate_hz`` (Poisson onsets) or ``n_firings`` (that many onsets,
    uniform) is given.  Onsets of one cascade are kept more than the
    cascade's largest span apart so firings never interleave."""
    neurons = list(neurons)
    span = sum(h for (_, h) in intervals)
    limit = duration_ticks - span - 1
    if limit <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64)
    if n_firings is None:
        T_s = duration_ticks / (1000.0 * TICKS_PER_MS)
        n_firings = rng.poisson(rate_hz * T_s)
    onsets = np.sort(np.floor(rng.random(int(n_firings)) * limit).astype(np.int64))
    keep = []
    last = None
    for o in onsets:
        if last is None or o - last > span:
            keep.append(o)
            last = o
    onsets = np.asarray(keep, np.int64)
    k = onsets.size
    ids = np.empty((k, len(neurons)), np.int64)
    ticks = np.empty((k, len(neurons)), np.int64)
    ids[:, 0] = neurons[0]
    ticks[:, 0] = onsets
    for j, (lo, hi) in enumerate(intervals):
        delay = rng.integers(lo + 1, hi + 1, size=k)
        ticks[:, j + 1] = ticks[:, j] + delay
        ids[:, j + 1] = neurons[j + 1]
    return ids.ravel(), ticks.ravel(), onsets


def _cascade_spec(rng, n_neurons, length, interval_set, neuron_pool=None):
    pool = np.arange(n_neurons) if neuron_pool is None else np.asarray(neuron_pool)
    neurons = [int(x) for x in rng.choice(pool, size=length, replace=False)]
    ivs = [interval_set[int(rng.integers(len(interval_set)))] for _ in range(length - 1)]
    return neurons, ivs


def make_stream(tag, n_neurons, rates_hz, duration_s, cascades, run=0):
    """Background + cascades.  ``cascades`` is a list of dicts with keys
    ``neurons``, ``intervals`` and one of ``rate_hz`` / ``n_firings``.
    Returns a dict with ids, ticks, num_types, duration_ticks and the
    cascades annotated with their planted onset count."""
    rng = rng_for(tag, run)
    dur = int(round(duration_s * 1000 * TICKS_PER_MS))
    if np.isscalar(rates_hz):
        rates_hz = np.full(n_neurons, float(rates_hz))
    parts_i, parts_t = [], []
    bi, bt = background(rng, rates_hz, dur)
    parts_i.append(bi)
    parts_t.append(bt)
    out_c = []
    for c in cascades:
        ci, ct, on = cascade_firings(rng, c["neurons"], c["intervals"], dur,
                                     rate_hz=c.get("rate_hz"),
                                     n_firings=c.get("n_firings"))
        parts_i.append(ci)
        parts_t.append(ct)
        cc = dict(c)
        cc["firings"] = int(on.size)
        out_c.append(cc)
    ids, ticks = sort_events(np.concatenate(parts_i), np.concatenate(parts_t))
    return {"ids": ids, "ticks": ticks, "num_types": int(n_neurons),
            "duration_ticks": dur, "cascades": out_c}


# --------------------------------------------------------------------------
# candidate tables: types[M, nmax] (-1 padded), len[M], lo/hi[M, nmax-1]
# --------------------------------------------------------------------------

def pack(episodes, nmax=None):
    M = len(episodes)
    if nmax is None:
        nmax = max([len(e[0]) for e in episodes] + [1])
    T = np.full((M, nmax), -1, np.int32)
    Ln = np.zeros(M, np.int32)
    LO = np.zeros((M, max(nmax - 1, 1)), np.int32)[:, :max(nmax - 1, 0)]
    HI = np.zeros((M, max(nmax - 1, 1)), np.int32)[:, :max(nmax - 1, 0)]
    LO = np.ascontiguousarray(LO)
    HI = np.ascontiguousarray(HI)
    for m, (ty, lo, hi) in enumerate(episodes):
        N = len(ty)
        T[m, :N] = ty
        Ln[m] = N
        if N > 1:
            LO[m, :N - 1] = lo
            HI[m, :N - 1] = hi
    return {"types": T, "len": Ln, "lo": LO, "hi": HI, "nmax": nmax, "M": M}


def sub_episodes(cascade, length):
    """Every contiguous sub-episode of a planted cascade with ``length``
    nodes, with the planted intervals."""
    nz, ivs = cascade["neurons"], cascade["intervals"]
    out = []
    for s in range(len(nz) - length + 1):
        iv = ivs[s:s + length - 1]
        out.append((tuple(nz[s:s + length]), tuple(l for l, _ in iv),
                    tuple(h for _, h in iv)))
    return out


def random_episodes(rng, M, n_types, N, interval_set, n_min=None):
    """M random episodes with N nodes (or N drawn from [n_min, N])."""
    if M <= 0:
        return []
    ks = np.full(M, N) if n_min is None else rng.integers(n_min, N + 1, size=M)
    ty = rng.integers(0, n_types, size=(M, N))
    iv = rng.integers(0, len(interval_set), size=(M, max(N - 1, 1)))
    los = np.array([a for a, _ in interval_set])
    his = np.array([b for _, b in interval_set])
    out = []
    for m in range(M):
        k = int(ks[m])
        out.append((tuple(int(x) for x in ty[m, :k]),
                    tuple(int(x) for x in los[iv[m, :k - 1]]),
                    tuple(int(x) for x in his[iv[m, :k - 1]])))
    return out


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config_plain(run=0):
    """Plain single stream: 64 neurons at 15 Hz for 20 s, two 4-node
    cascades firing 100 times each with hop delays in (2, 5] ms; candidates
    are all 4096 two-node episodes with (0, 5] ms; threshold 50."""
    tag = 1
    rng = rng_for(tag, 1000 + run)
    cascades = []
    used = rng.choice(64, size=8, replace=False)
    for c in range(2):
        cascades.append({"neurons": [int(x) for x in used[4 * c:4 * c + 4]],
                         "intervals": [(20, 50)] * 3, "n_firings": 100})
    s = make_stream(tag, 64, 15.0, 20.0, cascades, run)
    eps = [((a, b), (0,), (50,)) for a in range(64) for b in range(64)]
    s["candidates"] = pack(eps)
    s["theta"] = 50
    s["name"] = "plain: 64 neurons x 15 Hz x 20 s, 4096 two-node episodes (0,5] ms"
    return s


def config_mining(run=0, n_neurons=64, rate_hz=20.0, duration_s=780.0,
                  n_cascades=8, tag=2):
    """Level-wise mining stream: 64 neurons at 20 Hz for 780 s (about 1M
    events), eight cascades of 3-6 nodes firing at 1-3 Hz with hops drawn
    from {(0,5], (5,10], (10,20]} ms; threshold 0.5 Hz x duration, levels
    2-6.  Smaller variants (same recipe) serve as oracle-sized cases."""
    rng = rng_for(tag, 1000 + run)
    cascades = []
    for _ in range(n_cascades):
        L = int(rng.integers(3, 7))
        L = min(L, n_neurons)
        nz, ivs = _cascade_spec(rng, n_neurons, L, INTERVALS)
        cascades.append({"neurons": nz, "intervals": ivs,
                         "rate_hz": float(rng.uniform(1.0, 3.0))})
    s = make_stream(tag, n_neurons, rate_hz, duration_s, cascades, run)
    s["intervals"] = list(INTERVALS)
    s["theta"] = int(math.ceil(0.5 * duration_s))
    s["max_level"] = 6
    s["name"] = ("mining: %d neurons x %g Hz x %g s, %d cascades, levels 2-6"
                 % (n_neurons, rate_hz, duration_s, n_cascades))
    return s


def config_large(run=0, n_events=10_000_000, M_per_set=100_000, tag=3):
    """Large array: 256 neurons with log-normal rates (mean 10 Hz), about
    1e7 events, 32 cascades of 3-8 nodes; two candidate sets of 1e5
    episodes (N=3 and N=4): every planted contiguous sub-episode of that
    size, the rest random types and random intervals."""
    rng = rng_for(tag, 1000 + run)
    n_neurons = 256
    rates = rng.lognormal(mean=math.log(10.0) - 0.5, sigma=1.0, size=n_neurons)
    duration_s = n_events / rates.sum()
    cascades = []
    for _ in range(32):
        L = int(rng.integers(3, 9))
        nz, ivs = _cascade_spec(rng, n_neurons, L, INTERVALS)
        cascades.append({"neurons": nz, "intervals": ivs,
                         "rate_hz": float(rng.uniform(1.0, 3.0))})
    s = make_stream(tag, n_neurons, rates, duration_s, cascades, run)
    sets = {}
    for N in (3, 4):
        eps = []
        for c in cascades:
            eps.extend(sub_episodes(c, N))
        eps = eps[:M_per_set]
        eps.extend(random_episodes(rng, M_per_set - len(eps), n_neurons, N, INTERVALS))
        sets[N] = pack(eps)
    s["candidate_sets"] = sets
    s["theta"] = int(math.ceil(0.5 * duration_s))
    s["name"] = "large: 256 neurons, %d events, 2 x %d candidates (N=3, N=4)" % (
        s["ids"].size, M_per_set)
    return s


def config_batched(run=0, R=64, n_lo=1e4, n_hi=1e6, m_lo=1e3, m_hi=5e4, tag=4):
    """Batched: R recordings of uneven length (n log-uniform in [1e4, 1e6]),
    16-256 neurons at 20 Hz, 2-4 cascades of 2-8 nodes; each recording has
    its own candidate set (M log-uniform in [1e3, 5e4], N in 2..8, intervals
    from the set, planted sub-episodes included); threshold 0.5 Hz x T."""
    rng = rng_for(tag, 1000 + run)
    recs = []
    for r in range(R):
        n_target = float(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))
        nn = int(rng.integers(16, 257))
        rate = 20.0
        dur = n_target / (nn * rate)
        cascades = []
        for _ in range(int(rng.integers(2, 5))):
            L = int(rng.integers(2, 9))
            nz, ivs = _cascade_spec(rng, nn, L, INTERVALS)
            cascades.append({"neurons": nz, "intervals": ivs,
                             "rate_hz": float(rng.uniform(1.0, 3.0))})
        s = make_stream(tag * 1000 + r, nn, rate, dur, cascades, run)
        M = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        eps = []
        for c in cascades:
            for L in range(2, len(c["neurons"]) + 1):
                eps.extend(sub_episodes(c, L))
        eps = eps[:M]
        eps.extend(random_episodes(rng, M - len(eps), nn, 8, INTERVALS, n_min=2))
        s["candidates"] = pack(eps, nmax=8)
        s["theta"] = int(math.ceil(0.5 * dur))
        recs.append(s)
    return recs


def config_served(run=0, n_arrays=32, rate_req=200.0, trace_s=60.0,
                  M=50_000, preroll_s=60.0, win_lo_s=1.0, win_hi_s=60.0, tag=5):
    """Served: n_arrays simulated arrays (64-256 neurons at 20 Hz, four
    cascades on ids < 64 each) stream events; window-mining requests arrive
    as a Poisson process (rate_req per second in total, uniform array,
    window log-uniform in [1, 60] s); all requests are counted against one
    resident set of M episodes (N in 2..6, types < 64, planted
    sub-episodes included); threshold 0.5 Hz x window."""
    rng = rng_for(tag, 1000 + run)
    total_s = preroll_s + trace_s
    arrays = []
    all_casc = []
    for a in range(n_arrays):
        nn = int(rng.integers(64, 257))
        cascades = []
        for _ in range(4):
            L = int(rng.integers(2, 7))
            nz, ivs = _cascade_spec(rng, nn, L, INTERVALS, neuron_pool=np.arange(64))
            cascades.append({"neurons": nz, "intervals": ivs,
                             "rate_hz": float(rng.uniform(1.0, 3.0))})
        s = make_stream(tag * 1000 + a, nn, 20.0, total_s, cascades, run)
        arrays.append(s)
        all_casc.extend(cascades)
    eps = []
    for c in all_casc:
        for L in range(2, len(c["neurons"]) + 1):
            eps.extend(sub_episodes(c, L))
    eps = list(dict.fromkeys(eps))[:M]
    eps.extend(random_episodes(rng, M - len(eps), 64, 6, INTERVALS, n_min=2))
    n_req = int(rng.poisson(rate_req * trace_s))
    arrivals = np.sort(rng.random(n_req) * trace_s)
    req = []
    for k in range(n_req):
        a = int(rng.integers(n_arrays))
        w = float(math.exp(rng.uniform(math.log(win_lo_s), math.log(win_hi_s))))
        t_end = int(round((preroll_s + arrivals[k]) * 1000 * TICKS_PER_MS))
        t_begin = max(0, t_end - int(round(w * 1000 * TICKS_PER_MS)))
        req.append({"array": a, "t_begin": t_begin, "t_end": t_end,
                    "theta": int(math.ceil(0.5 * w)), "arrival_s": float(arrivals[k])})
    return {"arrays": arrays, "candidates": pack(eps, nmax=6), "requests": req,
            "preroll_s": preroll_s, "trace_s": trace_s}


def tiny_stream(rng, n, n_types, max_gap):
    """A short random stream with many ties (gaps drawn from 0..max_gap)."""
    ids = rng.integers(0, n_types, size=n).astype(np.int32)
    gaps = rng.integers(0, max_gap + 1, size=n)
    ticks = np.cumsum(gaps).astype(np.int32)
    return ids, ticks
