/* Sanitizer build (ASan + UBSan) of the CPU oracle, run over random streams
 * with ties: the projection mode against the full scan, the latest-only
 * relaxed counter (Algorithm 3) against the full-list one (the Observation
 * of Sec. 5.3.1), the two-pass pipeline (Algorithm 4) against separate
 * counts, the bound upper >= exact (Theorem of Sec. 5.3.2), and the
 * rejection of bad inputs. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_count_many(const int32_t *ids, const int32_t *ticks, int64_t n, int32_t num_types,
                   const int32_t *types, const int32_t *len, const int32_t *lo,
                   const int32_t *hi, int64_t M, int32_t nmax, int32_t mode,
                   int32_t projection, int32_t nthreads, int64_t *counts_out);
int64_t orc_two_pass(const int32_t *ids, const int32_t *ticks, int64_t n, int32_t num_types,
                     const int32_t *types, const int32_t *len, const int32_t *lo,
                     const int32_t *hi, int64_t M, int32_t nmax, int64_t theta,
                     int32_t projection, int32_t nthreads, int64_t *upper_out,
                     int64_t *exact_out);

static unsigned rng = 2463534242u;
static unsigned rnd(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 17;
    rng ^= rng << 5;
    return rng;
}

int main(void)
{
    enum { NMAX = 5, M = 300 };
    static int32_t types[M * NMAX], len[M], lo[M * (NMAX - 1)], hi[M * (NMAX - 1)];
    static int64_t a[M], b[M], up[M], ex[M];
    int fails = 0;
    for (int trial = 0; trial < 200; ++trial) {
        const int T = 2 + trial % 4;
        const int64_t n = rnd() % 400;
        int32_t *ids = malloc((size_t)(n ? n : 1) * sizeof(int32_t));
        int32_t *ticks = malloc((size_t)(n ? n : 1) * sizeof(int32_t));
        int32_t t = 0;
        for (int64_t i = 0; i < n; ++i) {
            t += (int32_t)(rnd() % 4);
            ids[i] = (int32_t)(rnd() % T);
            ticks[i] = t;
        }
        for (int m = 0; m < M; ++m) {
            len[m] = 1 + (int32_t)(rnd() % NMAX);
            for (int k = 0; k < NMAX; ++k) types[m * NMAX + k] = k < len[m] ? (int32_t)(rnd() % T) : -1;
            for (int k = 0; k < NMAX - 1; ++k) {
                const int32_t l = (int32_t)(rnd() % 6);
                lo[m * (NMAX - 1) + k] = l;
                hi[m * (NMAX - 1) + k] = l + 1 + (int32_t)(rnd() % 8);
            }
        }
        for (int mode = 0; mode < 3; ++mode) {
            if (orc_count_many(ids, ticks, n, T, types, len, lo, hi, M, NMAX, mode, 0, 2, a) ||
                orc_count_many(ids, ticks, n, T, types, len, lo, hi, M, NMAX, mode, 1, 3, b)) {
                fprintf(stderr, "count failed\n");
                return 1;
            }
            if (memcmp(a, b, sizeof a)) ++fails, fprintf(stderr, "projection differs (mode %d)\n", mode);
        }
        orc_count_many(ids, ticks, n, T, types, len, lo, hi, M, NMAX, 1, 0, 1, a);
        orc_count_many(ids, ticks, n, T, types, len, lo, hi, M, NMAX, 2, 0, 1, b);
        if (memcmp(a, b, sizeof a)) ++fails, fprintf(stderr, "latest-only differs from lists\n");
        const int64_t theta = 1 + trial % 5;
        const int64_t ns = orc_two_pass(ids, ticks, n, T, types, len, lo, hi, M, NMAX, theta,
                                        trial % 2, 2, up, ex);
        orc_count_many(ids, ticks, n, T, types, len, lo, hi, M, NMAX, 0, 0, 1, b);
        int64_t kept = 0;
        for (int m = 0; m < M; ++m) {
            if (up[m] != a[m]) ++fails, fprintf(stderr, "two-pass upper differs\n");
            if (up[m] >= theta) {
                ++kept;
                if (ex[m] != b[m]) ++fails, fprintf(stderr, "two-pass exact differs\n");
            } else if (ex[m] != -1) {
                ++fails, fprintf(stderr, "pruned candidate not -1\n");
            }
            if (b[m] > a[m]) ++fails, fprintf(stderr, "exact above relaxed\n");
        }
        if (kept != ns) ++fails, fprintf(stderr, "survivor count differs\n");
        free(ids);
        free(ticks);
    }
    /* bad inputs are refused */
    int32_t one = 0, bad_id = 9;
    int64_t c;
    if (orc_count_many(&bad_id, &one, 1, 2, types, len, lo, hi, 1, NMAX, 0, 1, 1, &c) != -1)
        ++fails, fprintf(stderr, "id out of range accepted\n");
    if (orc_count_many(&one, &one, 1, 2, types, len, lo, hi, 1, 9, 0, 0, 1, &c) != -1)
        ++fails, fprintf(stderr, "nmax out of range accepted\n");
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle: all checks passed\n");
    return 0;
}
