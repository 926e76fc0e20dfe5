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
