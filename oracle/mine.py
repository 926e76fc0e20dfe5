"""Level-wise mining for Problem 1 -- TEST INFRASTRUCTURE ONLY.

Problem 1 (Sec. 2): given an event stream, a set I of inter-event intervals
(t_low, t_high] and a threshold theta, find every serial episode whose hops
take intervals from I and whose non-overlapped count is >= theta.  The paper
mines level by level (Sec. 3, Sec. 5 intro): candidates of size l are
generated on the host from the frequent episodes of size l-1, counted, and
the frequent ones kept.  Counting each level uses Algorithm 4 (Sec. 5.3.2):
relaxed pass, elimination below theta, exact pass on the survivors.

The paper does not state the candidate-generation rule.  This oracle uses
the reading listed in the design notes:

* level 1: every event type, counted as its number of events (a 1-node
  episode occurs at each event of its type);
* level 2: every ordered pair (A, B) of frequent types, A == B allowed,
  times every interval of I;
* level l >= 3: alpha + beta's last node, for alpha, beta in F_(l-1) whose
  overlap agrees (alpha without its first node equals beta without its last
  node, types and intervals).  Restricting a set of non-overlapped
  occurrences to a prefix or suffix keeps them non-overlapped, so a frequent
  episode always has a frequent prefix and suffix.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from . import pack_candidates, two_pass


def gen_level2(F1, intervals):
    out = []
    for a in F1:
        for b in F1:
            for (l, h) in intervals:
                out.append(((a, b), (l,), (h,)))
    return out


def gen_next(F_prev):
    """Join F_(l-1) with itself on the (l-2)-node overlap (reading above)."""
    by_prefix = defaultdict(list)
    for (ty, lo, hi) in F_prev:
        by_prefix[(ty[:-1], lo[:-1], hi[:-1])].append((ty, lo, hi))
    out = []
    for (ty, lo, hi) in F_prev:
        key = (ty[1:], lo[1:], hi[1:])
        for (ty2, lo2, hi2) in by_prefix.get(key, ()):
            out.append((ty + ty2[-1:], lo + lo2[-1:], hi + hi2[-1:]))
    return out


def mine(ids, ticks, num_types, intervals, theta, max_level, projection=True,
         nthreads=0):
    """Returns {level: {"candidates": [...], "upper": int64[], "exact":
    int64[], "frequent": {episode: exact}}} for levels 1..max_level (stops
    early when a level has no candidates).  An episode is (types, lo, hi)
    tuples; ``intervals`` is a list of (lo, hi) in ticks."""
    ids = np.asarray(ids, np.int32)
    ticks = np.asarray(ticks, np.int32)
    result = {}
    hist = np.bincount(ids, minlength=num_types).astype(np.int64)
    cands = [((e,), (), ()) for e in range(num_types)]
    freq = {c: int(hist[c[0][0]]) for c in cands if hist[c[0][0]] >= theta}
    result[1] = {"candidates": cands, "upper": hist.copy(), "exact": hist.copy(),
                 "frequent": freq}
    F_prev = sorted(freq)
    for level in range(2, max_level + 1):
        if level == 2:
            cands = gen_level2([c[0][0] for c in F_prev], intervals)
        else:
            cands = gen_next(F_prev)
        if not cands:
            break
        T, Ln, LO, HI, _ = pack_candidates(cands)
        up, ex = two_pass(ids, ticks, num_types, T, Ln, LO, HI, theta,
                          projection=projection, nthreads=nthreads)
        freq = {c: int(x) for c, x in zip(cands, ex) if x >= theta}
        result[level] = {"candidates": cands, "upper": up, "exact": ex,
                         "frequent": freq}
        F_prev = sorted(freq)
        if not F_prev:
            break
    return result


# ---------------------------------------------------------------- array form
# The same generation rule and order as gen_level2 / gen_next above, on numpy
# arrays, for levels too large for Python tuples (millions of candidates).
# An episode set is (types [F, l], lo [F, l-1], hi [F, l-1]), int32.

def _rows(types, lo, hi):
    """One row per episode in tuple order: types..., lo..., hi... ."""
    return np.concatenate([types, lo, hi], axis=1)


def sort_episodes(types, lo, hi):
    """The episodes in Python's sorted() order of (types, lo, hi) tuples."""
    rows = _rows(types, lo, hi)
    order = np.lexsort(rows.T[::-1]) if rows.shape[0] else np.zeros(0, np.int64)
    return types[order], lo[order], hi[order]


def gen_level2_arrays(F1, intervals):
    """gen_level2 as arrays: a-major, then b, then the interval index."""
    F1 = np.asarray(F1, np.int32)
    I = np.asarray(intervals, np.int32).reshape(-1, 2)
    a, b, k = np.meshgrid(np.arange(F1.size), np.arange(F1.size), np.arange(I.shape[0]),
                          indexing="ij")
    a, b, k = a.ravel(), b.ravel(), k.ravel()
    types = np.stack([F1[a], F1[b]], axis=1).astype(np.int32)
    return types, I[k, :1].copy(), I[k, 1:].copy()


def gen_next_arrays(types, lo, hi):
    """gen_next as arrays: for each alpha in the given order, every beta (in
    the given order) whose first l-2 nodes and intervals equal alpha's last
    l-2, giving alpha + beta's last node and interval."""
    F, l = types.shape
    if F == 0:
        return (np.zeros((0, l + 1), np.int32), np.zeros((0, l), np.int32),
                np.zeros((0, l), np.int32))
    pre = _rows(types[:, :-1], lo[:, :-1], hi[:, :-1])   # beta's overlap key
    suf = _rows(types[:, 1:], lo[:, 1:], hi[:, 1:])      # alpha's overlap key
    # group the betas by key (stable, so each group keeps the given order)
    border = np.lexsort(pre.T[::-1]) if pre.shape[1] else np.arange(F)
    pk = pre[border]
    if pk.shape[1]:
        new = np.ones(F, bool)
        new[1:] = (pk[1:] != pk[:-1]).any(axis=1)
    else:
        new = np.zeros(F, bool)
        new[0] = True
    gstart = np.nonzero(new)[0]
    gend = np.append(gstart[1:], F)
    ukeys = pk[gstart]
    # each alpha's group: position of its suffix key among the unique keys
    def as_void(a):
        a = np.ascontiguousarray(a.astype(np.int64))
        return a.view(np.dtype((np.void, a.dtype.itemsize * a.shape[1]))).ravel()
    if ukeys.shape[1]:
        uo = np.lexsort(ukeys.T[::-1])   # already sorted; kept for clarity
        uv = as_void(ukeys[uo])
        sv = as_void(suf)
        pos = np.searchsorted(uv, sv)
        pos = np.minimum(pos, uv.size - 1)
        hit = uv[pos] == sv
        g = np.where(hit, uo[pos], -1)
    else:
        g = np.zeros(F, np.int64)
    cnt = np.where(g >= 0, gend[np.maximum(g, 0)] - gstart[np.maximum(g, 0)], 0)
    total = int(cnt.sum())
    alpha = np.repeat(np.arange(F), cnt)
    off = np.repeat(np.cumsum(cnt) - cnt, cnt)
    within = np.arange(total) - off
    beta = border[np.repeat(gstart[np.maximum(g, 0)], cnt) + within]
    t = np.concatenate([types[alpha], types[beta, -1:]], axis=1)
    a = np.concatenate([lo[alpha], lo[beta, -1:]], axis=1)
    b = np.concatenate([hi[alpha], hi[beta, -1:]], axis=1)
    return t.astype(np.int32), a.astype(np.int32), b.astype(np.int32)


def mine_arrays(ids, ticks, num_types, intervals, theta, max_level, nthreads=0,
                keep=None, planted=None, on_level=None):
    """mine() in array form (projection mode).  Per level: n_candidates,
    n_survivors (upper >= theta) and the frequent set (sorted) with its
    relaxed and exact counts.  keep(level, M) may ask for more: True = every
    candidate in generation order with its relaxed count and its exact count
    (of every candidate, pruned ones included: all_*); an index array = those
    candidates, plus every candidate equal to a row of planted(level) (rows
    types..., lo..., hi...), likewise (sample_*).  on_level(level, info) is
    called as each level completes."""
    from . import count, MODE_EXACT, MODE_RELAXED
    ids = np.asarray(ids, np.int32)
    ticks = np.asarray(ticks, np.int32)
    out = {}
    hist = np.bincount(ids, minlength=num_types).astype(np.int64)
    F1 = np.nonzero(hist >= theta)[0].astype(np.int32)
    out[1] = {"n_candidates": num_types, "n_survivors": num_types,
              "types": F1[:, None], "lo": np.zeros((F1.size, 0), np.int32),
              "hi": np.zeros((F1.size, 0), np.int32), "upper": hist[F1], "exact": hist[F1]}
    Ft, Fl, Fh = out[1]["types"], out[1]["lo"], out[1]["hi"]
    for level in range(2, max_level + 1):
        if level == 2:
            ct, cl, ch = gen_level2_arrays(F1, intervals)
        else:
            ct, cl, ch = gen_next_arrays(Ft, Fl, Fh)
        M = ct.shape[0]
        if M == 0:
            break
        Ln = np.full(M, level, np.int32)

        def exact_of(sel):
            return count(ids, ticks, num_types, ct[sel], Ln[sel], cl[sel], ch[sel], MODE_EXACT,
                         projection=True, nthreads=nthreads)
        up = count(ids, ticks, num_types, ct, Ln, cl, ch, MODE_RELAXED, projection=True,
                   nthreads=nthreads)
        surv = up >= theta
        want = keep(level, M) if keep else None
        info = {"n_candidates": M, "n_survivors": int(surv.sum())}
        ex = np.full(M, -1, np.int64)
        if want is True:
            ex_all = exact_of(slice(None))
            ex = np.where(surv, ex_all, -1)
            info.update({"all_types": ct, "all_lo": cl, "all_hi": ch, "all_upper": up,
                         "all_exact": ex_all})
        else:
            if surv.any():
                ex[surv] = exact_of(surv)
            if want is not None:
                idx = np.asarray(want, np.int64)
                if planted is not None:
                    prow = np.asarray(planted(level), np.int64)
                    if prow.shape[0]:
                        rows = _rows(ct, cl, ch).astype(np.int64)
                        v = np.dtype((np.void, 8 * rows.shape[1]))
                        rv = np.ascontiguousarray(rows).view(v).ravel()
                        pv = np.ascontiguousarray(prow).view(v).ravel()
                        idx = np.union1d(idx, np.nonzero(np.isin(rv, pv))[0])
                info.update({"sample_idx": idx, "sample_types": ct[idx], "sample_lo": cl[idx],
                             "sample_hi": ch[idx], "sample_upper": up[idx],
                             "sample_exact": exact_of(idx)})
        fr = ex >= theta
        Ft, Fl, Fh = sort_episodes(ct[fr], cl[fr], ch[fr])
        rows_f = _rows(ct[fr], cl[fr], ch[fr])
        order = np.lexsort(rows_f.T[::-1]) if rows_f.shape[0] else np.zeros(0, np.int64)
        info.update({"types": Ft, "lo": Fl, "hi": Fh, "upper": up[fr][order],
                     "exact": ex[fr][order]})
        out[level] = info
        if on_level:
            on_level(level, info)
        if Ft.shape[0] == 0:
            break
    return out
