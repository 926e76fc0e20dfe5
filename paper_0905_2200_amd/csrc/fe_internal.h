// fe_internal.h -- shared between the host runtime (fe_host.hip) and the
// device kernels (fe_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fe_const.h"

namespace fe {

// Per-key placement of candidate groups in the packed table.
struct Layout {
    int tile_base[NKEYS];  // first tile of the group
    int rec_base[NKEYS];   // int offset of the group's first record
};

// Everything a Map launch of one group needs.
struct MapGroup {
    const int *ids, *ticks;
    int n;
    const int *pk;     // group's first record
    const int *orig;   // [tiles*64] original candidate index, -1 = padding
    const int *lam;    // [tiles*(P+1)] look-back starts (P > 1)
    int2 *tbl;         // [P][tiles*64][KMAX] slot tables (P > 1)
    int *flags;        // [tiles*64] slot overflow flags (P > 1)
    int *out;          // [M] per original candidate
    int *status;
    const unsigned long long *cmask;  // type masks of aligned 8-event chunks, or null
    int tiles;
    int P;
    int sparse;  // shared-prefix waves use per-type dispatch
    int hashx;   // every type id is below 64: the type hash (id & 63) is the id
    int shlists; // exact, P = 1: waves of join siblings keep lists 0..N-3 once
};

// Batched counting (many recordings): one descriptor per recording and per
// packed tile, and the arguments of the persistent launches.
struct BJob {
    const int *ids, *ticks;
    int n;
    int theta;
    int *upper;  // relaxed counts [M_job]
    int *exact;  // exact counts [M_job], -1 for pruned
};

struct TileDesc {
    int job;      // recording
    int P;        // segments of the tile's group
    int otile;    // packed tile (record, orig and tileW index); may be shared
    int64_t rec;  // int offset of the tile record in pk
    int64_t tbl;  // int2 offset of the tile's slot tables [P][64][KMAX]
    int64_t lam;  // int offset of the tile's lam[P+1]
};

struct BatchDev {
    const TileDesc *tiles;
    const int2 *items;  // (tile, segment) work items, heaviest first
    int nitems;
    int *qctr;          // queue head
    const BJob *jobs;
    const int *pk;
    const int *orig;    // [tiles*64] candidate index within its recording
    int *lam;
    int2 *tbl;
    int *flags;
    int *status;
    int sparse;  // per-type dispatch for the bulk of each item
    int wpb;     // waves per block of the persistent launch (1..PERSIST_WPB_MAX)
};

// Exact count of candidates of the deep class: one wave per tile over the
// whole stream, each lane's N-1 lists as rings of `cap` windows in `ring`.
// A launch covers the group's flattened lanes [g0, g1) (lane index
// tile*64+lane, relative to pk/orig); ring holds (g1-g0)*(N-1)*cap windows.
struct DeepArgs {
    const int *ids, *ticks;
    int n;
    const int *pk;     // group's first record
    const int *orig;   // [tiles*64] candidate index, -1 = padding
    int64_t g0, g1;    // active lanes of this launch
    int2 *ring;
    int cap;
    int *out;          // [M] exact counts, by candidate index
    const int *upper;  // optional: lanes with upper[o] < theta write -1 (pruned)
    int theta;
    int from;                    // incremental count (count_io != null): events
    int *count_io, *last_io;     //   before `from` were counted by earlier calls
    int *status;
};
// window rings one deep launch may hold by default (bytes)
constexpr int64_t DEEP_SCRATCH = (int64_t)256 << 20;

constexpr int PERSIST_WPB_MAX = 8;

// launchers (fe_kernels.hip)
void launch_fill(int *p, int v, int64_t n, hipStream_t s);
void launch_validate(const int *ids, const int *ticks, int n, int num_types,
                     int *status, hipStream_t s);
void launch_prep_count(const int *types, const int *len, const int *lo,
                       const int *hi, int nmax, const int *sel,
                       const int *nsel, int M, int num_types, int exact,
                       int *keys, int *hist, int *status, int *bcnt, hipStream_t s);
// (bcnt: [NKEYS][(M + 255) / 256] per-block counts; boff: their exclusive
// scan, key-major)
void launch_prep_scatter(const int *types, const int *len, const int *lo,
                         const int *hi, int nmax, const int *sel,
                         const int *nsel, int M, const int *keys,
                         const Layout &lay, const int *boff, int *pk, int *orig,
                         int *tileW, hipStream_t s);
void launch_plan(const int *ticks, int n, const int *tileW, int tiles, int P,
                 int *lam, hipStream_t s);
void launch_map(int N, bool exact, int dcls, const MapGroup &g, hipStream_t s);
void launch_concat(const MapGroup &g, bool tree, hipStream_t s);
void launch_fixup(int N, bool exact, int dcls, const MapGroup &g, hipStream_t s);
void launch_persist(int N, bool exact, int dcls, const BatchDev &b, int grid, hipStream_t s);
void launch_resume(int N, bool exact, int dcls, const MapGroup &g, int from, int *count_io,
                   int *last_io, hipStream_t s);
void launch_deep(int N, const DeepArgs &a, hipStream_t s);
void launch_build_rec(const int *key, int m, const int *orig, int tiles, int *rec, int *tileW,
                      hipStream_t s);
// Run-aligned tiling of a level on the device (fe_tiling.hip).  scratch:
// tile_scratch_ints(M) ints; info: 5*NDCLS+1 ints (per class: tiles, first
// tile, run tiles, first run, candidates; then the total tiles).
int64_t tile_scratch_ints(int64_t M);
void launch_tile_plan(const int *key, int m, int64_t M, const int *up, int theta, bool exact,
                      int *scratch, int *info, hipStream_t s);
void launch_tile_lanes(int64_t M, const int *scratch, const int *info, int *orig, hipStream_t s);
// Join of sorted frequent m-node keys F into level m+1 keys (w = 3m-2;
// first/off from the host's range search), and a gather of selected keys.
void launch_join(const int *F, int w, const int64_t *first, const int64_t *off, int64_t cnt,
                 int64_t M, int *out, hipStream_t s);
void launch_gather_keys(const int *key, int w, const int *sel, int nsel, int *out, hipStream_t s);
// Sample of a level for the elimination decision: every SAMPLE_STRIDE-th
// block of 64 consecutive candidates; sample_count(M) candidates.
constexpr int SAMPLE_STRIDE = 64;
int64_t sample_count(int64_t M);
void launch_sample_keys(const int *key, int w, int64_t M, int *out, hipStream_t s);
// Exclusive scan of n ints (scratch: scan_scratch_ints(n) ints; its first
// holds the total).
int64_t scan_scratch_ints(int64_t n);
void launch_scan_excl(const int *in, int64_t n, int *out, int *scratch, hipStream_t s);
void launch_persist_fixup(int N, bool exact, int dcls, const BatchDev &b, const int *ctiles,
                          int nct, hipStream_t s);
void launch_plan_batch(const TileDesc *tiles, const BJob *jobs, const int *tileW,
                       const int *ptiles, int npt, int *lam, hipStream_t s);
void launch_clear_flags(const int *ptiles, int npt, int *fa, int *fb, hipStream_t s);
void launch_concat_batch(const BatchDev &b, const int *ctiles, int nct, bool exact,
                         hipStream_t s);
void launch_compact(const int *vals, int M, int theta, int *pruned_out,
                    int *sel, int *nsel, hipStream_t s);
void launch_select(const int *vals, const int *src, int M, int theta, int *out, hipStream_t s);
void launch_gather2(const int *a, const int *b, const int *sel, const int *nsel, int M,
                    int *out_a, int *out_b, hipStream_t s);
void launch_chunkmask(const int *ids, int n, unsigned long long *out, hipStream_t s);
void launch_histogram(const int *ids, int n, int num_types, int *hist,
                      hipStream_t s);

}  // namespace fe
