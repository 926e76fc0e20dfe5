/*
 * fe_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for counting non-overlapped
 * occurrences of serial episodes with inter-event delay constraints
 * (Cao et al., "Towards Chip-on-Chip Neuroscience: Fast Mining of Frequent
 * Episodes Using Graphics Processors").  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Every counting routine walks the event stream once, in stream order, per
 * candidate episode, exactly as the paper's serial counters do:
 *
 *   count_lists()   -- Algorithm 1 (Sec. 5.1, "Serial Episode Mining"):
 *                      one list of timestamps per episode node, scanned from
 *                      the newest entry to the oldest for a predecessor that
 *                      satisfies (t_low, t_high].  With relaxed != 0 the test
 *                      becomes 0 <= gap <= t_high, i.e. Algorithm 1 run on the
 *                      lower-bound-relaxed episode alpha' of Sec. 5.3.1 with
 *                      full lists (used to check the Observation of Sec. 5.3.1).
 *   count_latest()  -- Algorithm 3 (Sec. 5.3.1, "Less-Constrained Mining: A2"):
 *                      one timestamp per node, test gap <= t_high.
 *
 * Readings of the pseudocode (all listed in the design notes):
 *   - Completion happens at node i = N (Algorithm 1 prints |alpha|-1, which
 *     would make a 2-node episode uncountable; Algorithm 3 prints |alpha|).
 *   - The node loop runs from N down to 1, so an event is tested as a
 *     successor before it is pushed as a predecessor.
 *   - The relaxed constraint of A2 is the closed interval [0, t_high]: the
 *     printed check of Algorithm 3 has no lower bound at all.
 *   - An empty slot in Algorithm 3 never satisfies the check.
 *   - N = 1: every event of type E_(1) is an occurrence, so the count is the
 *     number of such events.
 *   - Stream order is semantic for equal timestamps; nothing is re-sorted.
 *   - In Algorithm 1's newest-to-oldest scan, entries are in non-decreasing
 *     time order, so once an entry is more than t_high older than t every
 *     older entry is too and the scan stops (it could never match).
 *
 * Integers only: ids and ticks are int32, counts are int64 internally.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_MODE_EXACT 0         /* Algorithm 1 with (lo, hi]             */
#define ORC_MODE_RELAXED 1       /* Algorithm 3 with [0, hi], latest only  */
#define ORC_MODE_RELAXED_LISTS 2 /* Algorithm 1 with [0, hi], full lists   */

#define ORC_NMAX 8

typedef struct {
    int32_t *v;
    int64_t len, cap;
} tlist;

static int tl_push(tlist *l, int32_t t)
{
    if (l->len == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 16;
        int32_t *nv = (int32_t *)realloc(l->v, (size_t)nc * sizeof(int32_t));
        if (!nv) return -1;
        l->v = nv;
        l->cap = nc;
    }
    l->v[l->len++] = t;
    return 0;
}

/*
 * Algorithm 1 (Sec. 5.1).  s[1..N-1] are the per-node lists (s[N] is never
 * read: a successful test at node N is a completion).  Event j is read as
 * (E, t) = (ids[idx[j]], ticks[idx[j]]) when idx is given (projection mode),
 * else (ids[j], ticks[j]).
 */
static int64_t count_lists(const int32_t *ids, const int32_t *ticks,
                           const int64_t *idx, int64_t n, const int32_t *E,
                           int N, const int32_t *lo, const int32_t *hi,
                           int relaxed)
{
    int64_t count = 0;
    if (N == 1) {
        for (int64_t j = 0; j < n; ++j) {
            int64_t q = idx ? idx[j] : j;
            if (ids[q] == E[0]) ++count;
        }
        return count;
    }
    tlist s[ORC_NMAX + 1];
    memset(s, 0, sizeof(s));
    for (int64_t j = 0; j < n; ++j) {
        int64_t q = idx ? idx[j] : j;
        int32_t e = ids[q];
        int32_t t = ticks[q];
        for (int i = N; i >= 1; --i) {
            if (e != E[i - 1]) continue;
            if (i == 1) {
                if (tl_push(&s[1], t)) goto oom;
                continue;
            }
            /* look in s[i-1] for t_prev with the constraint of hop i-1 */
            const int32_t l = lo[i - 2], h = hi[i - 2];
            int found = 0;
            for (int64_t k = s[i - 1].len - 1; k >= 0; --k) {
                int64_t d = (int64_t)t - (int64_t)s[i - 1].v[k];
                int ok = relaxed ? (d >= 0 && d <= h) : (d > l && d <= h);
                if (ok) { found = 1; break; }
                if (d > h) break;
            }
            if (!found) continue;
            if (i == N) {
                ++count;
                for (int k = 1; k <= N; ++k) s[k].len = 0;
                break; /* next event */
            }
            if (tl_push(&s[i], t)) goto oom;
        }
    }
    for (int k = 0; k <= N; ++k) free(s[k].v);
    return count;
oom:
    for (int k = 0; k <= N; ++k) free(s[k].v);
    return -1;
}

/* Algorithm 3 (Sec. 5.3.1): one timestamp per node, relaxed test gap <= hi. */
static int64_t count_latest(const int32_t *ids, const int32_t *ticks,
                            const int64_t *idx, int64_t n, const int32_t *E,
                            int N, const int32_t *hi)
{
    int64_t count = 0;
    if (N == 1) {
        for (int64_t j = 0; j < n; ++j) {
            int64_t q = idx ? idx[j] : j;
            if (ids[q] == E[0]) ++count;
        }
        return count;
    }
    int32_t s[ORC_NMAX + 1];
    int valid[ORC_NMAX + 1];
    for (int k = 0; k <= N; ++k) valid[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t q = idx ? idx[j] : j;
        int32_t e = ids[q];
        int32_t t = ticks[q];
        for (int i = N; i >= 1; --i) {
            if (e != E[i - 1]) continue;
            if (i == 1) {
                s[1] = t;
                valid[1] = 1;
                continue;
            }
            if (!valid[i - 1]) continue;
            if ((int64_t)t - (int64_t)s[i - 1] <= (int64_t)hi[i - 2]) {
                if (i == N) {
                    ++count;
                    for (int k = 0; k <= N; ++k) valid[k] = 0;
                    break;
                }
                s[i] = t;
                valid[i] = 1;
            }
        }
    }
    return count;
}

static int64_t count_one(const int32_t *ids, const int32_t *ticks,
                         const int64_t *idx, int64_t n, const int32_t *E,
                         int N, const int32_t *lo, const int32_t *hi, int mode)
{
    switch (mode) {
    case ORC_MODE_EXACT:
        return count_lists(ids, ticks, idx, n, E, N, lo, hi, 0);
    case ORC_MODE_RELAXED:
        return count_latest(ids, ticks, idx, n, E, N, hi);
    case ORC_MODE_RELAXED_LISTS:
        return count_lists(ids, ticks, idx, n, E, N, lo, hi, 1);
    default:
        return -2;
    }
}

/*
 * Projection: the sub-stream of events whose type belongs to the episode,
 * in stream order.  Removing events of other types changes no count, since
 * the counters above ignore them (the test suite checks this directly).
 * The merge walks per-type index lists (CSR by type) in index order.
 */
typedef struct {
    const int64_t *off; /* [num_types+1] */
    const int64_t *pos; /* [n] event indices grouped by type, ascending */
} type_index;

static int64_t project(const type_index *ti, const int32_t *E, int N,
                       int64_t *out)
{
    int32_t distinct[ORC_NMAX];
    int nd = 0;
    for (int i = 0; i < N; ++i) {
        int seen = 0;
        for (int k = 0; k < nd; ++k) seen |= (distinct[k] == E[i]);
        if (!seen) distinct[nd++] = E[i];
    }
    int64_t head[ORC_NMAX], end[ORC_NMAX];
    for (int k = 0; k < nd; ++k) {
        head[k] = ti->off[distinct[k]];
        end[k] = ti->off[distinct[k] + 1];
    }
    int64_t m = 0;
    for (;;) {
        int best = -1;
        for (int k = 0; k < nd; ++k)
            if (head[k] < end[k] &&
                (best < 0 || ti->pos[head[k]] < ti->pos[head[best]]))
                best = k;
        if (best < 0) break;
        out[m++] = ti->pos[head[best]++];
    }
    return m;
}

/*
 * Count M candidates.  types: [M*nmax] row-major (unused tail = -1),
 * len: [M], lo/hi: [M*(nmax-1)] row-major ticks.  counts_out: [M].
 * projection != 0 counts each candidate over its projected sub-stream.
 * nthreads <= 0 uses every available core.  Returns 0, or -1 on bad input /
 * out of memory.
 */
int orc_count_many(const int32_t *ids, const int32_t *ticks, int64_t n,
                   int32_t num_types, const int32_t *types, const int32_t *len,
                   const int32_t *lo, const int32_t *hi, int64_t M,
                   int32_t nmax, int32_t mode, int32_t projection,
                   int32_t nthreads, int64_t *counts_out)
{
    if (nmax < 1 || nmax > ORC_NMAX || M < 0 || n < 0) return -1;
    int64_t *off = NULL, *pos = NULL;
    type_index ti = {0, 0};
    if (projection) {
        if (num_types <= 0) return -1;
        off = (int64_t *)calloc((size_t)num_types + 1, sizeof(int64_t));
        pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int64_t *fill = (int64_t *)calloc((size_t)num_types + 1, sizeof(int64_t));
        if (!off || !pos || !fill) { free(off); free(pos); free(fill); return -1; }
        for (int64_t j = 0; j < n; ++j) {
            if (ids[j] < 0 || ids[j] >= num_types) { free(off); free(pos); free(fill); return -1; }
            off[ids[j] + 1]++;
        }
        for (int32_t k = 0; k < num_types; ++k) off[k + 1] += off[k];
        for (int64_t j = 0; j < n; ++j) pos[off[ids[j]] + fill[ids[j]]++] = j;
        free(fill);
        ti.off = off;
        ti.pos = pos;
    }
    int err = 0;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *buf = NULL;
        if (projection) buf = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        if (projection && !buf) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t m = 0; m < M; ++m) {
            if (err) continue;
            const int32_t *E = types + m * nmax;
            const int32_t N = len[m];
            if (N < 1 || N > nmax) {
#pragma omp atomic write
                err = 1;
                continue;
            }
            const int32_t *l = lo + m * (nmax - 1);
            const int32_t *h = hi + m * (nmax - 1);
            int64_t c;
            if (projection) {
                int bad = 0;
                for (int i = 0; i < N; ++i) bad |= (E[i] < 0 || E[i] >= num_types);
                if (bad) { c = 0; }
                else {
                    int64_t pn = project(&ti, E, N, buf);
                    c = count_one(ids, ticks, buf, pn, E, N, l, h, mode);
                }
            } else {
                c = count_one(ids, ticks, NULL, n, E, N, l, h, mode);
            }
            if (c < 0) {
#pragma omp atomic write
                err = 1;
            }
            counts_out[m] = c;
        }
        free(buf);
    }
    free(off);
    free(pos);
    return err ? -1 : 0;
}

/*
 * Algorithm 4 (Sec. 5.3.2, A2+A1): first pass counts the relaxed episode
 * alpha' with Algorithm 3; alpha is dropped when that count is below the
 * threshold; the second pass counts the survivors exactly with Algorithm 1.
 * upper_out[m] = A2 count; exact_out[m] = A1 count for survivors, -1 for
 * dropped candidates.  Returns the number of survivors, or -1 on error.
 */
int64_t orc_two_pass(const int32_t *ids, const int32_t *ticks, int64_t n,
                     int32_t num_types, const int32_t *types,
                     const int32_t *len, const int32_t *lo, const int32_t *hi,
                     int64_t M, int32_t nmax, int64_t theta,
                     int32_t projection, int32_t nthreads, int64_t *upper_out,
                     int64_t *exact_out)
{
    if (orc_count_many(ids, ticks, n, num_types, types, len, lo, hi, M, nmax,
                       ORC_MODE_RELAXED, projection, nthreads, upper_out))
        return -1;
    int64_t ns = 0;
    for (int64_t m = 0; m < M; ++m) ns += (upper_out[m] >= theta);
    int64_t *sel = (int64_t *)malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int64_t));
    int32_t *st = (int32_t *)malloc((size_t)(ns > 0 ? ns : 1) * nmax * sizeof(int32_t));
    int32_t *sl = (int32_t *)malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int32_t));
    int32_t w = nmax > 1 ? nmax - 1 : 1;
    int32_t *slo = (int32_t *)malloc((size_t)(ns > 0 ? ns : 1) * w * sizeof(int32_t));
    int32_t *shi = (int32_t *)malloc((size_t)(ns > 0 ? ns : 1) * w * sizeof(int32_t));
    int64_t *sc = (int64_t *)malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int64_t));
    if (!sel || !st || !sl || !slo || !shi || !sc) {
        free(sel); free(st); free(sl); free(slo); free(shi); free(sc);
        return -1;
    }
    int64_t k = 0;
    for (int64_t m = 0; m < M; ++m) {
        exact_out[m] = -1;
        if (upper_out[m] < theta) continue;
        sel[k] = m;
        memcpy(st + k * nmax, types + m * nmax, (size_t)nmax * sizeof(int32_t));
        sl[k] = len[m];
        if (nmax > 1) {
            memcpy(slo + k * (nmax - 1), lo + m * (nmax - 1), (size_t)(nmax - 1) * sizeof(int32_t));
            memcpy(shi + k * (nmax - 1), hi + m * (nmax - 1), (size_t)(nmax - 1) * sizeof(int32_t));
        }
        ++k;
    }
    int rc = orc_count_many(ids, ticks, n, num_types, st, sl, slo, shi, ns,
                            nmax, ORC_MODE_EXACT, projection, nthreads, sc);
    if (rc == 0)
        for (int64_t j = 0; j < ns; ++j) exact_out[sel[j]] = sc[j];
    free(sel); free(st); free(sl); free(slo); free(shi); free(sc);
    return rc ? -1 : ns;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
