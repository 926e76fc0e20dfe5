"""Brute force from the definitions -- TEST INFRASTRUCTURE ONLY.

Sec. 2 of the paper defines an occurrence of a serial episode with
inter-event constraints (each hop k satisfies t_low < t_(k+1) - t_(k) <=
t_high) and the frequency as the size of the largest set of non-overlapped
occurrences, two occurrences being non-overlapped when no event of one lies
between the events of the other.  On stream indices that is: the index spans
[i_1, i_N] of the two occurrences are disjoint.

This module enumerates every occurrence (index tuple) of an episode in a tiny
stream and computes the maximum number of pairwise disjoint spans twice, by
two unrelated methods:

* :func:`max_disjoint_exhaustive` -- search over subsets (branch and bound on
  the occurrence list), usable for a few dozen occurrences;
* :func:`max_disjoint_dp` -- dynamic programme over occurrences sorted by
  their last index: best[j] = max(best[j-1], 1 + best[last occurrence that
  ends before occurrence j starts]).

Neither uses the paper's counting algorithms.  ``relaxed=True`` uses the
relaxed constraint of Sec. 5.3.1 read as 0 <= gap <= t_high.
"""
from __future__ import annotations

import bisect
import itertools


def occurrences(ids, ticks, types, lo, hi, relaxed=False):
    """All index tuples i_1 < ... < i_N forming an occurrence."""
    n = len(ids)
    N = len(types)
    out = []

    def ok(k, a, b):
        d = ticks[b] - ticks[a]
        if relaxed:
            return 0 <= d <= hi[k]
        return lo[k] < d <= hi[k]

    def rec(prefix):
        k = len(prefix)
        if k == N:
            out.append(tuple(prefix))
            return
        start = prefix[-1] + 1 if prefix else 0
        for j in range(start, n):
            if ids[j] != types[k]:
                continue
            if k > 0 and not ok(k - 1, prefix[-1], j):
                continue
            prefix.append(j)
            rec(prefix)
            prefix.pop()

    rec([])
    return out


def _spans(occ):
    return sorted({(o[0], o[-1]) for o in occ}, key=lambda s: (s[1], s[0]))


def max_disjoint_exhaustive(occ):
    """Largest pairwise-disjoint subset of spans, by exhaustive search."""
    spans = _spans(occ)
    m = len(spans)
    best = 0

    def rec(i, chosen):
        nonlocal best
        if len(chosen) + (m - i) <= best:
            return
        if i == m:
            best = max(best, len(chosen))
            return
        a, b = spans[i]
        if all(b < c or d < a for (c, d) in chosen):
            chosen.append((a, b))
            rec(i + 1, chosen)
            chosen.pop()
        rec(i + 1, chosen)

    rec(0, [])
    return best


def max_disjoint_dp(occ):
    """Largest pairwise-disjoint subset of spans, by DP over span ends."""
    spans = _spans(occ)
    ends = [b for (_, b) in spans]
    best = [0] * (len(spans) + 1)
    for j, (a, b) in enumerate(spans, start=1):
        p = bisect.bisect_left(ends, a, 0, j - 1)  # spans ending strictly before a
        best[j] = max(best[j - 1], 1 + best[p])
    return best[-1]


def count(ids, ticks, types, lo, hi, relaxed=False, method="dp"):
    occ = occurrences(ids, ticks, types, lo, hi, relaxed)
    if method == "exhaustive":
        return max_disjoint_exhaustive(occ)
    return max_disjoint_dp(occ)


def all_streams(n, n_types, max_tick):
    """Every stream of length n over n_types with non-decreasing ticks in
    [0, max_tick] (ties in every order), as (ids, ticks) tuples."""
    for ticks in itertools.combinations_with_replacement(range(max_tick + 1), n):
        for ids in itertools.product(range(n_types), repeat=n):
            yield list(ids), list(ticks)
