/*
 * fe.h -- C ABI of the MI355X frequent-episode counting library (libfe.so).
 *
 * The library counts non-overlapped occurrences of serial episodes with
 * inter-event delay constraints over one time-ordered event stream, the
 * problem of Sec. 2 of Cao et al., "Towards Chip-on-Chip Neuroscience: Fast
 * Mining of Frequent Episodes Using Graphics Processors":
 *
 *   - an event stream is n events (E_i, t_i) with t_i <= t_(i+1) (Sec. 2,
 *     first definition); here E_i is an int32 event type (a neuron id) in
 *     [0, num_types) and t_i an int32 tick in [0, 2^30);
 *   - a serial episode is an ordered tuple of N event types with one delay
 *     interval (lo_k, hi_k] per hop, k = 1..N-1 (Sec. 2, second definition
 *     and the inter-event constraint inequalities); types may repeat;
 *   - its count is the size of the largest set of non-overlapped
 *     occurrences (Sec. 2, "frequency of episodes"), computed by the serial
 *     state machine of Algorithm 1 (Sec. 5.1);
 *   - the relaxed count drops the lower bounds (Sec. 5.3.1, Algorithm 3): a
 *     hop is satisfied by 0 <= gap <= hi_k; it is an upper bound on the
 *     count (Theorem of Sec. 5.3.2);
 *   - Problem 1 (Sec. 2): every episode with hops drawn from an interval set
 *     I whose count is >= theta, mined level by level (Sec. 5 intro).
 *
 * Conventions for every call
 *   - Return value: FE_OK (0) or a positive fe_status code.  Host-checkable
 *     argument errors return at once and enqueue nothing.
 *   - Pointers named "device" are HIP device pointers (e.g. torch CUDA
 *     tensors' data_ptr()).  The caller owns them and keeps them valid
 *     until the enqueued work has finished (fe_sync, or a synchronisation
 *     of the context's stream).
 *   - Work is enqueued on the context's stream.  Calls that need a size
 *     known only on the device (candidate grouping, survivor counts, mining
 *     levels) synchronise that stream internally before returning; they say
 *     so below.
 *   - Stream checks (sortedness, id and tick ranges) and candidate checks
 *     run on the device.  A violation makes the call return FE_EUNSORTED,
 *     FE_ERANGE or FE_EINVAL; no output is written in that case.
 *   - The library owns its workspace (grown on demand, freed by
 *     fe_destroy).  One context must not be used from two host threads at
 *     once.
 *
 * Candidate table (device, row-major, int32):
 *   types[M * nmax]       E_(1..N) of candidate m in types[m*nmax + 0..N-1],
 *                         the rest unused;
 *   len[M]                N of candidate m, 1 <= N <= nmax <= 8;
 *   lo[M * (nmax-1)]      lo_k of hop k in lo[m*(nmax-1) + k], k < N-1;
 *   hi[M * (nmax-1)]      hi_k likewise.  0 <= lo_k < hi_k < 2^30 and
 *                         sum_k hi_k < 2^30.
 *   Every such hop is counted exactly.  Algorithm 1's list for hop k matters
 *   only through the ticks that pass its test, a union of windows of which
 *   at most hi_k/(hi_k-lo_k+1)+1 are live at once.  Candidates whose hops
 *   all have at most 8 live windows keep their lists in registers; the
 *   others (narrow intervals far from 0, e.g. (190,200] ticks) keep them as
 *   rings in library-owned device memory, min(bound, n) windows per list,
 *   and are counted over the whole stream by a kernel of their own.  If one
 *   candidate's rings cannot be allocated the call returns FE_ENOMEM.
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fe_status {
    FE_OK = 0,
    FE_EINVAL = 1,    /* bad argument or candidate                          */
    FE_ENOMEM = 2,    /* device or host allocation failed                   */
    FE_EDEVICE = 3,   /* a HIP runtime call failed                          */
    FE_EUNSORTED = 4, /* stream ticks decrease somewhere                    */
    FE_ERANGE = 5,    /* an id outside [0,num_types) or tick outside [0,2^30) */
    FE_EBUSY = 6,     /* server request not finished yet                    */
    FE_EINTERNAL = 7  /* an internal invariant failed (a library bug)       */
} fe_status;

typedef enum fe_mode {
    FE_EXACT = 0,  /* Algorithm 1: hop constraint lo < gap <= hi            */
    FE_RELAXED = 1 /* Algorithm 3: hop constraint 0 <= gap <= hi (lo unused) */
} fe_mode;

/* Tunables for fe_set_param. */
typedef enum fe_param {
    FE_PARAM_SEGMENTS = 0,   /* MapConcatenate segment count P; 0 = automatic  */
    FE_PARAM_TARGET_WAVES = 1, /* waves the automatic P aims for per launch
                                (default 16384: two generations of 8 waves
                                per SIMD on 256 CUs)                          */
    FE_PARAM_MIN_SEG_EVENTS = 2, /* smallest segment the automatic P allows   */
    FE_PARAM_CONCAT_TREE = 3, /* 1 = wave-shuffle tree Concatenate when P >= 16,
                                 0 = per-candidate sequential walk             */
    FE_PARAM_TIMING = 4,     /* 1 = time every kernel launch with HIP events on
                                the context's stream (fe_get_kernel_stats)     */
    FE_PARAM_TYPE_DISPATCH = 5, /* 1 (default) = per-type dispatch: a lane steps
                                only the events of its own episode's types
                                (for waves whose candidates share their first
                                N-1 types, those events wave-wide plus each
                                lane's own last-type events); 0 = every event
                                through every lane.  Read at each count call,
                                at fe_batch_create and at each server round.
                                Counts are identical either way.              */
    FE_PARAM_CROSSOVER_A = 6, /* hybrid rule (Algorithm 2, Eq. 2), exact       */
    FE_PARAM_CROSSOVER_B = 7, /* counter: a group of tiles >= A/N + B tiles of
                                N-node candidates is counted whole-stream
                                (P = 1), a smaller one by MapConcatenate with
                                P >= 2.  Defaults 8472 and 13112 (A may be
                                negative): the least-squares fit to crossovers
                                measured on a 256-CU MI355X (python -m
                                paper_0905_2200_amd.crossover).  Ignored when
                                FE_PARAM_SEGMENTS > 0.                        */
    FE_PARAM_ELIMINATION = 8, /* fe_mine, per level: 1 = two-pass elimination
                                (Algorithm 4: relaxed pass, prune, exact pass
                                on the survivors); 0 = one pass of Algorithm 1
                                over every candidate (upper reported as -1);
                                2 (default) = decided per level: levels of
                                fewer than FE_PARAM_SAMPLE_MIN candidates take
                                two passes; for larger ones the relaxed pass
                                first runs on a sample (every 64th block of 64
                                consecutive candidates) and two passes are
                                taken when the sampled survivor fraction s
                                satisfies s < 1 - FE_PARAM_PASS1_COST/1000
                                (then the relaxed pass costs less than it
                                saves), else one; with FE_PARAM_PASS1_COST
                                >= 1000 no sample is taken and such levels
                                take one pass.  The frequent episodes and
                                exact counts are the same either way.          */
    FE_PARAM_HOST_TILING = 9, /* fe_mine: 0 (default) = each level's
                                candidates are pruned and tiled on the device
                                (sibling runs whole, by list-depth class);
                                1 = the same tiling on the host (the relaxed
                                counts are copied back and the lane assignment
                                uploaded).  Same tiles, same results.  The
                                per-level decision of FE_PARAM_ELIMINATION = 2
                                needs device tiling; with host tiling it takes
                                two passes.                                    */
    FE_PARAM_KEEP_CANDIDATES = 10, /* fe_mine: 1 = also return every
                                candidate of each level with its counts
                                (fe_level.all_*); 0 (default) = the frequent
                                episodes only                                  */
    FE_PARAM_CROSSOVER_A_RELAXED = 11, /* the hybrid rule's A and B for the  */
    FE_PARAM_CROSSOVER_B_RELAXED = 12, /* relaxed counter (Algorithm 3);
                                defaults 9699 and 6165 (same fit)             */
    FE_PARAM_PASS1_COST = 13, /* cost of the relaxed pass per candidate, in
                                thousandths of the exact pass's (default
                                1000: on the mining workload's level 4 the
                                relaxed pass takes as long as the exact one
                                with shared lists); used by
                                FE_PARAM_ELIMINATION = 2                      */
    FE_PARAM_SAMPLE_MIN = 14, /* smallest level sampled by FE_PARAM_ELIMINATION
                                = 2 (default 131072 candidates)                */
    FE_PARAM_SHARED_LISTS = 15 /* 1 (default) = exact whole-stream counting of
                                a tile whose candidates share every node but
                                the last and every hop but the last (join
                                siblings, N >= 3) keeps lists 0..N-3 once per
                                tile, each entry with the start index of its
                                newest chain; 0 = per-candidate lists (same
                                counts)                                       */
} fe_param;

typedef struct fe_ctx fe_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is the
 * hipStream_t all work is enqueued on (NULL: the device's null stream,
 * which is also what torch reports for its default stream). */
int fe_create(int device, void *hip_stream, fe_ctx **out);

/* Synchronise, free all workspace and the context. */
int fe_destroy(fe_ctx *ctx);

/* Message for the last error of this context (static storage of ctx). */
const char *fe_last_error(const fe_ctx *ctx);

/* Wait for the context's stream; return the first error detected on the
 * device since the last fe_sync (and clear it), else FE_OK. */
int fe_sync(fe_ctx *ctx);

/* Set a tunable (fe_param).  Values < 0 are rejected. */
int fe_set_param(fe_ctx *ctx, int param, int64_t value);
int fe_get_param(const fe_ctx *ctx, int param, int64_t *value);

/* Check a stream (device ids[n], ticks[n]) on the device: ticks
 * non-decreasing, 0 <= tick < 2^30, 0 <= id < num_types.  Synchronises;
 * returns FE_OK, FE_EUNSORTED or FE_ERANGE. */
int fe_validate(fe_ctx *ctx, const int32_t *ids, const int32_t *ticks,
                int64_t n, int32_t num_types);

/* Count every candidate over the stream (Algorithm 1 for FE_EXACT,
 * Algorithm 3 for FE_RELAXED), by MapConcatenate over P index segments
 * (Sec. 5.2.2) with exact segment stitching.  counts_out: device int32[M],
 * in candidate order.  Synchronises once (candidate grouping). */
int fe_count(fe_ctx *ctx, const int32_t *ids, const int32_t *ticks, int64_t n,
             int32_t num_types, const int32_t *types, const int32_t *len,
             const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax,
             int mode, int32_t *counts_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fe_count
 * with the same arguments, semantics and results, whose workspace (candidate
 * grouping, packed tiles, segment tables, window rings) is carved from a
 * fixed 64 MiB device array that the library holds on each device until the
 * process ends.  It calls no hipMalloc, hipFree or allocating library
 * routine (the context's pinned staging and status word, made by
 * fe_create, are reused).  Limit: inputs whose whole-stream workspace
 * (about 4 B per candidate, (3*nmax-2)*4 B per candidate for the packed
 * table, and 1 B per event) exceeds 64 MiB are rejected with FE_ENOMEM
 * before any work is enqueued; the segment count is lowered until the
 * segment tables fit what is left.  Every call on one device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device -- from any context -- race, so order them (e.g. one stream, or
 * fe_sync between them).  FE_EDEVICE if the array could not be located on
 * the device at fe_create.  Synchronises once (candidate grouping). */
int fe_count_noalloc(fe_ctx *ctx, const int32_t *ids, const int32_t *ticks, int64_t n,
                     int32_t num_types, const int32_t *types, const int32_t *len,
                     const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax,
                     int mode, int32_t *counts_out);

/* Incremental counting of a growing recording, processed in consecutive
 * partitions (the paper's real-time "chip-on-chip" use, Sec. 1 and Sec. 7).
 * ids/ticks[0, n) on the device are the stream so far; the events before
 * `from` must be the ones earlier calls saw (append-only).  count_io and
 * last_io (device int32[M], in candidate order) carry, per candidate, the
 * completions counted in [0, from) and the index of the last of them (-1 if
 * none); on return they cover [0, n).  Start with 0 / -1 / from = 0, then
 * call with from = the previous n after each append.  The counts equal
 * fe_count over [0, n) in the same mode.  Why it is exact: after a
 * completion the machine is empty, and no occurrence spans more than
 * W = sum(hi) ticks, so from `from` on the machine acts like a fresh one
 * started after max(last, lam-1), lam = first index with tick >= t_from - W
 * (the argument behind the segment stitching of fe_count); only that much
 * is read again before `from`.  Errors: FE_EINVAL for from outside [0, n],
 * null carry arrays or bad candidates (as fe_count); stream errors as
 * fe_validate.  Synchronises once (candidate grouping). */
int fe_count_resume(fe_ctx *ctx, const int32_t *ids, const int32_t *ticks, int64_t n,
                    int32_t num_types, const int32_t *types, const int32_t *len,
                    const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax,
                    int mode, int64_t from, int32_t *count_io, int32_t *last_io);

/* Two-pass elimination, Algorithm 4 (Sec. 5.3.2): upper_out[m] = relaxed
 * count; candidates with upper < theta are dropped (exact_out[m] = -1);
 * exact_out[m] = exact count for the others.  *n_survivors_out (device
 * int32) receives the number kept.  All outputs are device pointers.
 * Synchronises (grouping of each pass). */
int fe_count_two_pass(fe_ctx *ctx, const int32_t *ids, const int32_t *ticks,
                      int64_t n, int32_t num_types, const int32_t *types,
                      const int32_t *len, const int32_t *lo,
                      const int32_t *hi, int32_t M, int32_t nmax,
                      int32_t theta, int32_t *upper_out, int32_t *exact_out,
                      int32_t *n_survivors_out);

/* ---------------------------------------------------------------- mining */

typedef struct fe_level {
    int32_t level;        /* episode size N                                 */
    int64_t n_candidates; /* candidates counted at this level               */
    int64_t n_survivors;  /* candidates kept by the relaxed pass            */
    int64_t n_frequent;   /* candidates whose exact count >= theta          */
    int32_t *types;       /* [n_frequent * level] frequent episodes, sorted  */
    int32_t *lo;          /* [n_frequent * (level-1)]                       */
    int32_t *hi;          /* [n_frequent * (level-1)]                       */
    int32_t *upper;       /* [n_frequent] relaxed counts                    */
    int32_t *exact;       /* [n_frequent] exact counts                      */
    double gen_ms;        /* host candidate generation time                 */
    double count_ms;      /* device counting time (both passes)             */
    int32_t passes;       /* 2: relaxed pass, elimination, exact pass on the
                             survivors (Algorithm 4); 1: exact pass only
                             (upper = -1, n_survivors = n_candidates)       */
    int64_t sample_n;     /* candidates of the relaxed sample that decided
                             the level's passes (0: none was taken)         */
    int64_t sample_kept;  /* of which survived (upper >= theta)             */
    /* With FE_PARAM_KEEP_CANDIDATES = 1, every candidate of the level in
     * generation order (n_candidates entries each; NULL otherwise): */
    int32_t *all_types;   /* [n_candidates * level]                         */
    int32_t *all_lo;      /* [n_candidates * (level-1)]                     */
    int32_t *all_hi;      /* [n_candidates * (level-1)]                     */
    int32_t *all_upper;   /* relaxed counts, -1 in a one-pass level         */
    int32_t *all_exact;   /* exact counts, -1 where the relaxed pass pruned */
} fe_level;

typedef struct fe_result {
    int32_t n_levels;
    fe_level *levels;     /* levels[0] is level 1 */
} fe_result;

/* Problem 1 (Sec. 2) by level-wise mining.  Level 1 counts each event type
 * (a 1-node episode occurs at every event of its type); level 2 takes every
 * ordered pair of frequent types (repeats allowed) times every interval of
 * I; level l >= 3 joins two frequent (l-1)-node episodes whose overlapping
 * l-2 nodes and intervals agree.  Every level is counted with Algorithm 4
 * on the device; generation runs on the host (Sec. 5 intro).  Stops after
 * max_level or at the first level with no frequent episode.  ids, ticks:
 * device; iv_lo, iv_hi: host int32[n_iv] (the set I, in ticks).
 * *out is allocated by the library; free it with fe_result_free.
 * Synchronises. */
int fe_mine(fe_ctx *ctx, const int32_t *ids, const int32_t *ticks, int64_t n,
            int32_t num_types, const int32_t *iv_lo, const int32_t *iv_hi,
            int32_t n_iv, int32_t theta, int32_t max_level, fe_result **out);

void fe_result_free(fe_result *res);

/* ------------------------------------------------------------- batching */

/* One recording of a batch: its stream, its own candidate table (fe_count
 * layout, mixed episode sizes allowed), its threshold and its outputs.  All
 * pointers are device pointers owned by the caller. */
typedef struct fe_job {
    const int32_t *ids, *ticks;
    int64_t n;
    int32_t num_types;
    const int32_t *types, *len, *lo, *hi;
    int32_t M, nmax;
    int32_t theta;
    int32_t *upper_out; /* [M] relaxed counts (Algorithm 3)                   */
    int32_t *exact_out; /* [M] exact counts (Algorithm 1), -1 when pruned     */
} fe_job;

typedef struct fe_batch fe_batch;

/* Launch shape of a batch, picked by fe_batch_autotune or set by hand. */
typedef struct fe_batch_tuning {
    int32_t seg_events;   /* target events per work item (segment length)    */
    int32_t waves_per_cu; /* persistent waves launched per compute unit      */
    int32_t waves_per_block; /* work items (one per wave) per workgroup of the
                             persistent launches: 1, 2, 4 or 8 (0: 4)        */
    double run_ms;        /* measured duration of one fe_batch_run (autotune) */
} fe_batch_tuning;

/* Plan the two-pass count (Algorithm 4) of R recordings as one batch:
 * validates every stream and candidate table (synchronises), tiles every
 * recording's candidates, splits long recordings into MapConcatenate
 * segments, orders all (tile, segment) work items heaviest first, and
 * captures one HIP graph per episode size: a persistent relaxed launch over
 * every recording's items of that size, Concatenate, then a persistent
 * exact launch over the survivors and Concatenate.  The streams and
 * candidate tables must stay unchanged and valid while the batch exists. */
int fe_batch_create(fe_ctx *ctx, int32_t R, const fe_job *jobs, fe_batch **out);

/* Replay the batch's graphs on the context's stream (asynchronous). */
int fe_batch_run(fe_batch *b);

/* Time `reps` runs for each launch shape of a small grid (segment length x
 * persistent waves per CU x waves per workgroup), keep the fastest; *best
 * receives it.
 * Synchronises. */
int fe_batch_autotune(fe_batch *b, int32_t reps, fe_batch_tuning *best);
int fe_batch_set_tuning(fe_batch *b, const fe_batch_tuning *t);
int fe_batch_get_tuning(const fe_batch *b, fe_batch_tuning *t);
int fe_batch_destroy(fe_batch *b);

/* Convenience: create a batch, run it once, synchronise, destroy it. */
int fe_count_batched(fe_ctx *ctx, int32_t R, const fe_job *jobs);

/* -------------------------------------------------------------- serving */

/* A window-counting service over many device-resident event streams
 * ("arrays", e.g. one per multi-electrode array) and one resident candidate
 * set: each request asks for the two-pass count (Algorithm 4) of every
 * resident candidate over one array's events with ticks in
 * [t_begin, t_end).  This serves the paper's goal of processing partitions
 * of a live stream in turn (Sec. 1).  A scheduler thread inside the library
 * admits waiting requests into rounds while their summed device footprint
 * fits the per-round share of the HBM budget, and keeps up to max_inflight
 * rounds on the GPU at once (one stream each): requests that arrive while
 * others run join the next round as soon as a stream and memory free up. */
typedef struct fe_server fe_server;

typedef struct fe_server_config {
    int32_t n_arrays;      /* number of streams                               */
    int64_t capacity;      /* events each array's device buffer holds          */
    int64_t hbm_budget;    /* bytes of per-request device state in flight      */
    int32_t max_inflight;  /* rounds on the device at once (>= 1)              */
    int32_t max_round;     /* requests per round (>= 1)                        */
    int32_t seg_events;    /* target events per work item (0: 16384)           */
    int32_t waves_per_cu;  /* persistent waves per compute unit (0: 16)        */
} fe_server_config;

typedef struct fe_request {
    int32_t array;
    int32_t t_begin, t_end; /* window of ticks [t_begin, t_end)               */
    int32_t theta;          /* support threshold of this request              */
    int64_t arrival_ns;     /* caller's steady-clock arrival time; 0 = now    */
} fe_request;

typedef struct fe_response {
    int32_t status;         /* FE_OK, or why the request failed               */
    int32_t n_events;       /* events in the window                           */
    int32_t n_survivors;    /* candidates kept by the relaxed pass            */
    int32_t n_frequent;     /* candidates with exact count >= theta           */
    const int32_t *upper;   /* [M] host, valid until fe_server_release        */
    const int32_t *exact;   /* [M] host, -1 for pruned candidates             */
    int64_t arrival_ns, admit_ns, done_ns; /* steady clock (ns)               */
    int32_t round, round_size;             /* the round it ran in, its size   */
    int64_t footprint;      /* device bytes the request needed in its round   */
} fe_response;

typedef struct fe_server_stats {
    int64_t submitted, completed, rejected, rounds;
    int32_t largest_round, max_inflight_seen;
    int64_t budget_closed;  /* rounds closed because the next waiting request
                               did not fit the round's share of hbm_budget   */
} fe_server_stats;

/* Create a server: the resident candidates (device table, fe_count layout)
 * are checked and packed once; num_types is a host array [n_arrays]. */
int fe_server_create(fe_ctx *ctx, const fe_server_config *cfg, const int32_t *num_types,
                     const int32_t *types, const int32_t *len, const int32_t *lo,
                     const int32_t *hi, int32_t M, int32_t nmax, fe_server **out);

/* Append n events (host arrays, sorted, not earlier than the array's last
 * event, ids in range) to an array's device buffer.  FE_ENOMEM when the
 * buffer would overflow. */
int fe_server_append(fe_server *s, int32_t array, const int32_t *ids, const int32_t *ticks,
                     int64_t n);

/* Queue a request; *ticket identifies it. */
int fe_server_submit(fe_server *s, const fe_request *req, uint64_t *ticket);

/* FE_EBUSY while the request is queued or running; FE_OK with *out filled
 * once it is done (out->status tells whether it succeeded). */
int fe_server_poll(fe_server *s, uint64_t ticket, fe_response *out);

/* Block until the request is done, then as fe_server_poll. */
int fe_server_wait(fe_server *s, uint64_t ticket, fe_response *out);

/* Forget a finished request and free its host results. */
int fe_server_release(fe_server *s, uint64_t ticket);

int fe_server_get_stats(fe_server *s, fe_server_stats *out);

/* Stop the scheduler (finishing the rounds in flight) and free everything. */
int fe_server_destroy(fe_server *s);

/* Per-call statistics of the last fe_count / fe_count_two_pass / fe_mine
 * call on this context (host memory owned by ctx). */
typedef struct fe_stats {
    int64_t map_launches;   /* Map kernel launches                          */
    int64_t segments_max;   /* largest P used                               */
    int64_t fallback_cands; /* candidates recounted over the whole stream
                               because a look-back held too many slots      */
    double last_call_ms;    /* host wall time of the last call              */
} fe_stats;

int fe_get_stats(const fe_ctx *ctx, fe_stats *out);

/* Per-kernel timing (FE_PARAM_TIMING = 1): for each kernel kind, the number
 * of launches, their summed and largest duration measured with HIP events
 * recorded around each launch on the context's stream, and the algorithmic
 * work they did in candidate-episode x event units (candidates counted x
 * stream events; 0 for kernels that do not scan the stream). */
typedef struct fe_kernel_stat {
    char name[40];
    int64_t launches;
    double total_ms;
    double max_ms;
    double ee;
} fe_kernel_stat;

/* Copies up to cap entries into out, sets *n_out to the number of kinds.
 * Synchronises the context's stream. */
int fe_get_kernel_stats(fe_ctx *ctx, fe_kernel_stat *out, int32_t cap, int32_t *n_out);
int fe_reset_kernel_stats(fe_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
