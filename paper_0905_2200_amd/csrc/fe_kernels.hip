// fe_kernels.hip -- utility kernels (fill, stream validation, candidate
// grouping, segment plan, Concatenate, elimination, level-1 histogram) and
// the dispatch of the per-N Map kernels (fe_map.h, fe_map_n<N>.hip).
#include "fe_internal.h"

namespace fe {

__device__ __forceinline__ int uniform_u(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------------ utilities
__global__ void k_fill(int *p, int v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill(int *p, int v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

// ------------------------------------------------------------------ validate
__global__ void k_validate(const int *__restrict__ ids, const int *__restrict__ ticks,
                           int n, int num_types, int *status)
{
    int bits = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int e = ids[i], t = ticks[i];
        if (e < 0 || e >= num_types || t < 0 || t >= TICK_LIMIT) bits |= ST_RANGE;
        if (i > 0 && ticks[i - 1] > t) bits |= ST_UNSORTED;
    }
    if (bits) atomicOr(status, bits);
}

void launch_validate(const int *ids, const int *ticks, int n, int num_types, int *status,
                     hipStream_t s)
{
    if (n <= 0) return;
    int blocks = (n + 1023) / 1024;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, s, ids, ticks, n, num_types,
                       status);
}

// ------------------------------------------------------------------ candidate grouping
// Key of a candidate: (N-1)*NDCLS + list-depth class (0 for the relaxed
// counter); -1 if the candidate is invalid.  W_out: sum of hi; B_out: the
// largest window bound of its hops (the ring capacity of the deep class).
__device__ int cand_key(const int *types, const int *len, const int *lo, const int *hi,
                        int nmax, int m, int num_types, int exact, int *W_out, int *B_out)
{
    const int N = len[m];
    if (N < 1 || N > nmax) return -1;
    const int64_t tb = (int64_t)m * nmax, ib = (int64_t)m * (nmax - 1);
    for (int k = 0; k < N; ++k) {
        const int t = types[tb + k];
        if (t < 0 || t >= num_types) return -1;
    }
    int64_t W = 0;
    int bound = 1;
    for (int k = 0; k < N - 1; ++k) {
        const int l = lo[ib + k], h = hi[ib + k];
        if (l < 0 || l >= h || h >= TICK_LIMIT) return -1;
        W += h;
        const int b = window_bound(l, h);
        bound = b > bound ? b : bound;
    }
    if (W >= TICK_LIMIT) return -1;
    *W_out = (int)W;
    *B_out = bound;
    return (N - 1) * NDCLS + (exact ? depth_class(bound) : 0);
}

// Wave-aggregated "reserve one slot in counter[key]" -- returns the rank of
// this lane among lanes of the wave with the same key plus the counter's old
// value.  Lanes with key < 0 do nothing and get -1.
__device__ int wave_reserve(int key, int *counter)
{
    const int lane = __lane_id();
    bool pending = key >= 0;
    int pos = -1;
    for (;;) {
        const unsigned long long act = __ballot(pending);
        if (act == 0) break;
        const int leader = __ffsll((long long)act) - 1;
        const int k0 = __shfl(key, leader);
        const bool mine = pending && key == k0;
        const unsigned long long mask = __ballot(mine);
        if (mine) {
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            int base = 0;
            if (lane == leader) base = atomicAdd(&counter[k0], __popcll(mask));
            base = __shfl(base, leader);
            pos = base + rank;
            pending = false;
        }
    }
    return pos;
}

// hist[key] += candidates with that key; hist[NKEYS + key] = max W among
// them; hist[2*NKEYS + key] = their largest window bound; bcnt[key * nb +
// block] = the block's candidates with that key.
__global__ void k_prep_count(const int *types, const int *len, const int *lo, const int *hi,
                             int nmax, const int *sel, const int *nsel, int M, int num_types,
                             int exact, int *keys, int *hist, int *status, int *bcnt, int nb)
{
    __shared__ int sc[NKEYS];
    if (threadIdx.x < NKEYS) sc[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = __lane_id();
    const int lim = nsel ? *nsel : M;
    int key = -1, W = 0, B = 1;
    if (i < lim) {
        const int m = sel ? sel[i] : i;
        key = cand_key(types, len, lo, hi, nmax, m, num_types, exact, &W, &B);
        if (key < 0) atomicOr(status, ST_BADCAND);
        keys[i] = key;
    }
    bool pending = key >= 0;
    for (;;) {
        const unsigned long long act = __ballot(pending);
        if (act == 0) break;
        const int leader = __ffsll((long long)act) - 1;
        const int k0 = __shfl(key, leader);
        const bool mine = pending && key == k0;
        int wm = mine ? W : 0, bm = mine ? B : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const int o = __shfl_xor(wm, off), ob = __shfl_xor(bm, off);
            wm = o > wm ? o : wm;
            bm = ob > bm ? ob : bm;
        }
        const int cntk = __popcll(__ballot(mine));
        if (lane == leader) {
            atomicAdd(&hist[k0], cntk);
            atomicMax(&hist[NKEYS + k0], wm);
            atomicMax(&hist[2 * NKEYS + k0], bm);
            atomicAdd(&sc[k0], cntk);
        }
        pending = pending && !mine;
    }
    __syncthreads();
    if (threadIdx.x < NKEYS) bcnt[(int64_t)threadIdx.x * nb + blockIdx.x] = sc[threadIdx.x];
}

void launch_prep_count(const int *types, const int *len, const int *lo, const int *hi, int nmax,
                       const int *sel, const int *nsel, int M, int num_types, int exact,
                       int *keys, int *hist, int *status, int *bcnt, hipStream_t s)
{
    if (M <= 0) return;
    const int nb = (M + 255) / 256;
    hipLaunchKernelGGL(k_prep_count, dim3(nb), dim3(256), 0, s, types, len, lo, hi, nmax, sel,
                       nsel, M, num_types, exact, keys, hist, status, bcnt, nb);
}

// Each candidate goes to its key group in input order: its rank is the
// group's candidates in earlier blocks (boff: exclusive scan of the per-block
// counts, key-major), then in earlier waves of the block, then in earlier
// lanes -- so runs of siblings given in order stay together.
__global__ void k_prep_scatter(const int *types, const int *len, const int *lo, const int *hi,
                               int nmax, const int *sel, const int *nsel, int M,
                               const int *keys, Layout lay, const int *boff, int nb, int *pk,
                               int *orig, int *tileW)
{
    constexpr int WV = 256 / WAVE;
    __shared__ int wc[WV][NKEYS];
    if (threadIdx.x < WV * NKEYS) (&wc[0][0])[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const int lim = nsel ? *nsel : M;
    const int key = i < lim ? keys[i] : -1;
    int rank = 0;
    bool pending = key >= 0;
    for (;;) {
        const unsigned long long act = __ballot(pending);
        if (act == 0) break;
        const int leader = __ffsll((long long)act) - 1;
        const int k0 = __shfl(key, leader);
        const bool mine = pending && key == k0;
        const unsigned long long mask = __ballot(mine);
        if (mine) rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == leader) wc[wv][k0] = __popcll(mask);
        pending = pending && !mine;
    }
    __syncthreads();
    if (key < 0) return;
    for (int w = 0; w < wv; ++w) rank += wc[w][key];
    const int r = boff[(int64_t)key * nb + blockIdx.x] - boff[(int64_t)key * nb] + rank;
    const int m = sel ? sel[i] : i;
    const int N = key / NDCLS + 1;
    const int tile = lay.tile_base[key] + r / WAVE;
    const int tl = r % WAVE;  // lane of the tile
    int *rec = pk + lay.rec_base[key] + (int64_t)(r / WAVE) * rec_ints(N);
    const int64_t tb = (int64_t)m * nmax, ib = (int64_t)m * (nmax - 1);
    int W = 0;
    for (int k = 0; k < N; ++k) rec[k * WAVE + tl] = types[tb + k];
    for (int k = 0; k < N - 1; ++k) {
        rec[(N + k) * WAVE + tl] = lo[ib + k];
        rec[(2 * N - 1 + k) * WAVE + tl] = hi[ib + k];
        W += hi[ib + k];
    }
    orig[(int64_t)tile * WAVE + tl] = m;
    atomicMax(&tileW[tile], W);
}

void launch_prep_scatter(const int *types, const int *len, const int *lo, const int *hi,
                         int nmax, const int *sel, const int *nsel, int M, const int *keys,
                         const Layout &lay, const int *boff, int *pk, int *orig, int *tileW,
                         hipStream_t s)
{
    if (M <= 0) return;
    const int nb = (M + 255) / 256;
    hipLaunchKernelGGL(k_prep_scatter, dim3(nb), dim3(256), 0, s, types, len, lo, hi, nmax, sel,
                       nsel, M, keys, lay, boff, nb, pk, orig, tileW);
}

// ------------------------------------------------------------------ segment plan
// lam[tile*(P+1)+p] = first index i with ticks[i] >= ticks[L_p] - W(tile),
// L_p = p*n/P; lam[.., 0] = 0 and lam[.., P] = n.
__global__ void k_plan(const int *__restrict__ ticks, int n, const int *__restrict__ tileW,
                       int tiles, int P, int *__restrict__ lam)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)tiles * (P + 1)) return;
    const int tile = (int)(i / (P + 1)), p = (int)(i % (P + 1));
    if (p == 0) { lam[i] = 0; return; }
    if (p == P) { lam[i] = n; return; }
    const int L = (int)((int64_t)p * n / P);
    const int x = ticks[L] - tileW[tile];
    int a = 0, b = L;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (ticks[mid] < x) a = mid + 1;
        else b = mid;
    }
    lam[i] = a;
}

void launch_plan(const int *ticks, int n, const int *tileW, int tiles, int P, int *lam,
                 hipStream_t s)
{
    const int64_t tot = (int64_t)tiles * (P + 1);
    hipLaunchKernelGGL(k_plan, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ticks, n,
                       tileW, tiles, P, lam);
}

// ------------------------------------------------------------------ Map dispatch
void launch_map_n1(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n2(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n3(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n4(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n5(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n6(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n7(bool, int, const MapGroup &, hipStream_t, bool);
void launch_map_n8(bool, int, const MapGroup &, hipStream_t, bool);

static void dispatch(int N, bool exact, int dcls, const MapGroup &g, hipStream_t s, bool fix)
{
    switch (N) {
    case 1: return launch_map_n1(exact, dcls, g, s, fix);
    case 2: return launch_map_n2(exact, dcls, g, s, fix);
    case 3: return launch_map_n3(exact, dcls, g, s, fix);
    case 4: return launch_map_n4(exact, dcls, g, s, fix);
    case 5: return launch_map_n5(exact, dcls, g, s, fix);
    case 6: return launch_map_n6(exact, dcls, g, s, fix);
    case 7: return launch_map_n7(exact, dcls, g, s, fix);
    default: return launch_map_n8(exact, dcls, g, s, fix);
    }
}

void launch_persist_n1(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n2(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n3(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n4(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n5(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n6(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n7(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);
void launch_persist_n8(bool, int, const BatchDev &, int, const int *, int, hipStream_t, bool);

static void pdispatch(int N, bool exact, int dcls, const BatchDev &b, int grid, const int *ct,
                      int nct, hipStream_t s, bool fix)
{
    switch (N) {
    case 1: return launch_persist_n1(exact, dcls, b, grid, ct, nct, s, fix);
    case 2: return launch_persist_n2(exact, dcls, b, grid, ct, nct, s, fix);
    case 3: return launch_persist_n3(exact, dcls, b, grid, ct, nct, s, fix);
    case 4: return launch_persist_n4(exact, dcls, b, grid, ct, nct, s, fix);
    case 5: return launch_persist_n5(exact, dcls, b, grid, ct, nct, s, fix);
    case 6: return launch_persist_n6(exact, dcls, b, grid, ct, nct, s, fix);
    case 7: return launch_persist_n7(exact, dcls, b, grid, ct, nct, s, fix);
    default: return launch_persist_n8(exact, dcls, b, grid, ct, nct, s, fix);
    }
}

void launch_resume_n1(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n2(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n3(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n4(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n5(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n6(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n7(bool, int, const MapGroup &, int, int *, int *, hipStream_t);
void launch_resume_n8(bool, int, const MapGroup &, int, int *, int *, hipStream_t);

void launch_deep_n1(const DeepArgs &, hipStream_t);
void launch_deep_n2(const DeepArgs &, hipStream_t);
void launch_deep_n3(const DeepArgs &, hipStream_t);
void launch_deep_n4(const DeepArgs &, hipStream_t);
void launch_deep_n5(const DeepArgs &, hipStream_t);
void launch_deep_n6(const DeepArgs &, hipStream_t);
void launch_deep_n7(const DeepArgs &, hipStream_t);
void launch_deep_n8(const DeepArgs &, hipStream_t);

void launch_deep(int N, const DeepArgs &a, hipStream_t s)
{
    switch (N) {
    case 1: return launch_deep_n1(a, s);
    case 2: return launch_deep_n2(a, s);
    case 3: return launch_deep_n3(a, s);
    case 4: return launch_deep_n4(a, s);
    case 5: return launch_deep_n5(a, s);
    case 6: return launch_deep_n6(a, s);
    case 7: return launch_deep_n7(a, s);
    default: return launch_deep_n8(a, s);
    }
}

void launch_resume(int N, bool exact, int dcls, const MapGroup &g, int from, int *count_io,
                   int *last_io, hipStream_t s)
{
    switch (N) {
    case 1: return launch_resume_n1(exact, dcls, g, from, count_io, last_io, s);
    case 2: return launch_resume_n2(exact, dcls, g, from, count_io, last_io, s);
    case 3: return launch_resume_n3(exact, dcls, g, from, count_io, last_io, s);
    case 4: return launch_resume_n4(exact, dcls, g, from, count_io, last_io, s);
    case 5: return launch_resume_n5(exact, dcls, g, from, count_io, last_io, s);
    case 6: return launch_resume_n6(exact, dcls, g, from, count_io, last_io, s);
    case 7: return launch_resume_n7(exact, dcls, g, from, count_io, last_io, s);
    default: return launch_resume_n8(exact, dcls, g, from, count_io, last_io, s);
    }
}

void launch_persist(int N, bool exact, int dcls, const BatchDev &b, int grid, hipStream_t s)
{
    pdispatch(N, exact, dcls, b, grid, nullptr, 0, s, false);
}

void launch_persist_fixup(int N, bool exact, int dcls, const BatchDev &b, const int *ctiles,
                          int nct, hipStream_t s)
{
    pdispatch(N, exact, dcls, b, 0, ctiles, nct, s, true);
}

// Look-back starts of every segmented tile of a batch: one wave per tile.
__global__ void k_plan_batch(const TileDesc *tiles, const BJob *jobs, const int *tileW,
                             const int *ptiles, int npt, int *lam)
{
    const int lane = __lane_id();
    const int w = uniform_u(blockIdx.x * WPB + (threadIdx.x >> 6));
    if (w >= npt) return;
    const int tile = ptiles[w];
    const TileDesc td = tiles[tile];
    const BJob jb = jobs[td.job];
    const int n = jb.n, P = td.P, W = tileW[td.otile];
    for (int p = lane; p <= P; p += WAVE) {
        int v;
        if (p == 0) {
            v = 0;
        } else if (p == P) {
            v = n;
        } else {
            const int L = (int)((int64_t)p * n / P);
            const int x = jb.ticks[L] - W;
            int a = 0, b = L;
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (jb.ticks[mid] < x) a = mid + 1;
                else b = mid;
            }
            v = a;
        }
        lam[td.lam + p] = v;
    }
}

void launch_plan_batch(const TileDesc *tiles, const BJob *jobs, const int *tileW,
                       const int *ptiles, int npt, int *lam, hipStream_t s)
{
    if (npt <= 0) return;
    hipLaunchKernelGGL(k_plan_batch, dim3((npt + WPB - 1) / WPB), dim3(WAVE * WPB), 0, s, tiles,
                       jobs, tileW, ptiles, npt, lam);
}

// Clear the slot-overflow flags of the listed tiles (both passes).
__global__ void k_clear_flags(const int *ptiles, int npt, int *fa, int *fb)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int w = g / WAVE, lane = g % WAVE;
    if (w >= npt) return;
    const int64_t c = (int64_t)ptiles[w] * WAVE + lane;
    fa[c] = 0;
    fb[c] = 0;
}

void launch_clear_flags(const int *ptiles, int npt, int *fa, int *fb, hipStream_t s)
{
    if (npt <= 0) return;
    const int64_t thr = (int64_t)npt * WAVE;
    hipLaunchKernelGGL(k_clear_flags, dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, s, ptiles,
                       npt, fa, fb);
}

__device__ __forceinline__ int clampk_b(int x) { return x < 0 ? 0 : (x >= KMAX ? KMAX - 1 : x); }

// Concatenate for every segmented tile of a batch: one lane per candidate
// walks its segments' slot tables.  Exact pass: pruned candidates get -1.
__global__ void k_concat_batch(BatchDev b, const int *ctiles, int nct, int exact)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int w = g / WAVE, lane = g % WAVE;
    if (w >= nct) return;
    const int tile = ctiles[w];
    const TileDesc td = b.tiles[tile];
    const BJob jb = b.jobs[td.job];
    const int c = tile * WAVE + lane;
    const int o = b.orig[(int64_t)td.otile * WAVE + lane];
    if (o < 0) return;
    int *out = exact ? jb.exact : jb.upper;
    if (exact && jb.upper[o] < jb.theta) {
        out[o] = -1;
        return;
    }
    if (b.flags[c]) return;
    const int2 *t = b.tbl + td.tbl;
    int x = 0, tot = 0;
    for (int p = 0; p < td.P; ++p) {
        const int2 v = t[((int64_t)p * WAVE + lane) * KMAX + x];
        tot += v.x;
        x = clampk_b(v.y);
    }
    out[o] = tot;
}

void launch_concat_batch(const BatchDev &b, const int *ctiles, int nct, bool exact, hipStream_t s)
{
    if (nct <= 0) return;
    const int64_t thr = (int64_t)nct * WAVE;
    hipLaunchKernelGGL(k_concat_batch, dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, s, b,
                       ctiles, nct, exact ? 1 : 0);
}

void launch_map(int N, bool exact, int dcls, const MapGroup &g, hipStream_t s)
{
    dispatch(N, exact, dcls, g, s, false);
}

void launch_fixup(int N, bool exact, int dcls, const MapGroup &g, hipStream_t s)
{
    dispatch(N, exact, dcls, g, s, true);
}

// ------------------------------------------------------------------ Concatenate
// (c, x) o (c', x')[sigma] = (c[sigma] + c'[x[sigma]], x'[x[sigma]]); the
// count is the composition over all segments applied to slot 0 of segment 0.
__device__ __forceinline__ int clampk(int x) { return x < 0 ? 0 : (x >= KMAX ? KMAX - 1 : x); }

__global__ void k_concat_seq(MapGroup g)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.tiles * WAVE) return;
    const int o = g.orig[c];
    if (o < 0 || g.flags[c]) return;
    const int64_t stride = (int64_t)g.tiles * WAVE * KMAX;
    const int2 *t = g.tbl + (int64_t)c * KMAX;
    int x = 0, tot = 0;
    for (int p = 0; p < g.P; ++p) {
        const int2 v = t[p * stride + x];
        tot += v.x;
        x = clampk(v.y);
    }
    g.out[o] = tot;
}

// One wave per candidate: lane l composes a contiguous chunk of segments
// sequentially, then the 64 chunk tables are composed pairwise in log2(64)
// steps through LDS (lane l takes lane l+s's table at the slot its own
// entries exit into).  Every wave of the block takes part in the barriers.
__global__ __launch_bounds__(WAVE *WPB) void k_concat_tree(MapGroup g)
{
    __shared__ int sc[WPB][WAVE][KMAX];
    __shared__ int sx[WPB][WAVE][KMAX];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const int c = uniform_u(blockIdx.x * WPB + wv);
    const bool have = c < g.tiles * WAVE && g.orig[c] >= 0 && !g.flags[c];
    const int P = g.P;
    const int cs = (P + WAVE - 1) / WAVE;
    const int p0 = lane * cs;
    const int p1 = p0 + cs < P ? p0 + cs : P;
    const int64_t stride = (int64_t)g.tiles * WAVE * KMAX;
    const int2 *t = g.tbl + (int64_t)(have ? c : 0) * KMAX;
    int tc[KMAX], tx[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        int x = j, tot = 0;
        if (have)
            for (int p = p0; p < p1; ++p) {
                const int2 v = t[p * stride + x];
                tot += v.x;
                x = clampk(v.y);
            }
        tc[j] = tot;
        tx[j] = x;
    }
    for (int s = 1; s < WAVE; s <<= 1) {
#pragma unroll
        for (int j = 0; j < KMAX; ++j) { sc[wv][lane][j] = tc[j]; sx[wv][lane][j] = tx[j]; }
        __syncthreads();
        if ((lane & (2 * s - 1)) == 0 && lane + s < WAVE) {
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                const int q = tx[j];
                tc[j] += sc[wv][lane + s][q];
                tx[j] = sx[wv][lane + s][q];
            }
        }
        __syncthreads();
    }
    if (have && lane == 0) g.out[g.orig[c]] = tc[0];
}

void launch_concat(const MapGroup &g, bool tree, hipStream_t s)
{
    const int cands = g.tiles * WAVE;
    if (tree)
        hipLaunchKernelGGL(k_concat_tree, dim3((cands + WPB - 1) / WPB), dim3(WAVE * WPB), 0, s, g);
    else
        hipLaunchKernelGGL(k_concat_seq, dim3((cands + 255) / 256), dim3(256), 0, s, g);
}

// ------------------------------------------------------------------ elimination
// Algorithm 4's elimination: keep m when vals[m] >= theta (appending m to
// sel), else write -1 into pruned_out[m].
__global__ void k_compact(const int *vals, int M, int theta, int *pruned_out, int *sel, int *nsel)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < M;
    const bool keep = in && vals[i] >= theta;
    if (in && !keep && pruned_out) pruned_out[i] = -1;
    const int r = wave_reserve(keep ? 0 : -1, nsel);
    if (keep) sel[r] = i;
}

void launch_compact(const int *vals, int M, int theta, int *pruned_out, int *sel, int *nsel,
                    hipStream_t s)
{
    if (M <= 0) return;
    hipLaunchKernelGGL(k_compact, dim3((M + 255) / 256), dim3(256), 0, s, vals, M, theta,
                       pruned_out, sel, nsel);
}

// out[m] = vals[m] >= theta ? src[m] : -1
__global__ void k_select(const int *vals, const int *src, int M, int theta, int *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[i] = vals[i] >= theta ? src[i] : -1;
}

void launch_select(const int *vals, const int *src, int M, int theta, int *out, hipStream_t s)
{
    if (M <= 0) return;
    hipLaunchKernelGGL(k_select, dim3((M + 255) / 256), dim3(256), 0, s, vals, src, M, theta, out);
}

// out_a[i] = a[sel[i]], out_b[i] = b[sel[i]] for i < *nsel
__global__ void k_gather2(const int *a, const int *b, const int *sel, const int *nsel, int *out_a,
                          int *out_b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *nsel) return;
    out_a[i] = a[sel[i]];
    out_b[i] = b[sel[i]];
}

void launch_gather2(const int *a, const int *b, const int *sel, const int *nsel, int M, int *out_a,
                    int *out_b, hipStream_t s)
{
    if (M <= 0) return;
    hipLaunchKernelGGL(k_gather2, dim3((M + 255) / 256), dim3(256), 0, s, a, b, sel, nsel, out_a,
                       out_b);
}

// Tile records of the mining driver, built on the device from the level's
// episode keys (3m-2 ints each, interleaved (E1, lo1, hi1, E2, ..., E_m))
// and the host's lane assignment orig[tile*64+lane] (-1 = padding): the
// same layout the device grouping writes.  tileW[tile] = largest sum(hi).
__global__ __launch_bounds__(WAVE *WPB) void k_build_rec(const int *__restrict__ key, int m,
                                                         const int *__restrict__ orig, int tiles,
                                                         int *__restrict__ rec,
                                                         int *__restrict__ tileW)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int t = blockIdx.x * WPB + (threadIdx.x >> 6);
    if (t >= tiles) return;
    const int idx = orig[(int64_t)t * WAVE + lane];
    int *r = rec + (int64_t)t * rec_ints(m);
    int W = 0;
    if (idx < 0) {
        for (int k = 0; k < m; ++k) r[k * WAVE + lane] = -1;
        for (int k = 0; k < m - 1; ++k) {
            r[(m + k) * WAVE + lane] = 0;
            r[(2 * m - 1 + k) * WAVE + lane] = 0;
        }
    } else {
        const int *kk = key + (int64_t)idx * (3 * m - 2);
        for (int k = 0; k < m; ++k) r[k * WAVE + lane] = kk[3 * k];
        for (int k = 0; k < m - 1; ++k) {
            const int hi = kk[3 * k + 2];
            r[(m + k) * WAVE + lane] = kk[3 * k + 1];
            r[(2 * m - 1 + k) * WAVE + lane] = hi;
            W += hi;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(W, off);
        W = o > W ? o : W;
    }
    if (lane == 0) tileW[t] = W;
}

void launch_build_rec(const int *key, int m, const int *orig, int tiles, int *rec, int *tileW,
                      hipStream_t s)
{
    if (tiles <= 0) return;
    hipLaunchKernelGGL(k_build_rec, dim3((unsigned)((tiles + WPB - 1) / WPB)), dim3(WAVE * WPB),
                       0, s, key, m, orig, tiles, rec, tileW);
}

// out[c] = OR over the events of chunk c (indices 8c..8c+7) of 1 << (id & 63)
__global__ void k_chunkmask(const int *__restrict__ ids, int n, unsigned long long *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c * 8 >= n) return;
    unsigned long long m = 0;
    const int e = c * 8 + 8 < n ? c * 8 + 8 : n;
    for (int i = c * 8; i < e; ++i) m |= 1ull << (ids[i] & 63);
    out[c] = m;
}

void launch_chunkmask(const int *ids, int n, unsigned long long *out, hipStream_t s)
{
    if (n <= 0) return;
    const int chunks = (n + 7) / 8;
    hipLaunchKernelGGL(k_chunkmask, dim3((chunks + 255) / 256), dim3(256), 0, s, ids, n, out);
}

// ------------------------------------------------------------------ level 1
__global__ void k_histogram(const int *__restrict__ ids, int n, int num_types, int *hist)
{
    extern __shared__ int sh[];
    const bool lds = num_types <= 8192;
    if (lds)
        for (int k = threadIdx.x; k < num_types; k += blockDim.x) sh[k] = 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int e = ids[i];
        if (e < 0 || e >= num_types) continue;
        if (lds) atomicAdd(&sh[e], 1);
        else atomicAdd(&hist[e], 1);
    }
    __syncthreads();
    if (lds)
        for (int k = threadIdx.x; k < num_types; k += blockDim.x)
            if (sh[k]) atomicAdd(&hist[k], sh[k]);
}

void launch_histogram(const int *ids, int n, int num_types, int *hist, hipStream_t s)
{
    if (n <= 0) return;
    int blocks = (n + 4095) / 4096;
    if (blocks > 1024) blocks = 1024;
    const size_t sh = num_types <= 8192 ? (size_t)num_types * sizeof(int) : 0;
    hipLaunchKernelGGL(k_histogram, dim3(blocks), dim3(256), sh, s, ids, n, num_types, hist);
}

}  // namespace fe
