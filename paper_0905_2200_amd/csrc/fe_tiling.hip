// Level-wise mining on the device: candidate generation by the join, and
// run-aligned tiling of a level's candidates for both passes of Algorithm 4.
//
// Input: the level's keys in generation order (per candidate t0 lo0 hi0 t1
// ... t_{m-1}) and, for the exact pass, the relaxed counts: the survivors are
// the candidates with upper >= theta (the elimination step), kept in
// generation order.  They are grouped by list-depth class (stable), and in
// each class cut into maximal runs of equal first m-1 types (join siblings).
// A run fills whole tiles; a remainder of at least half a tile gets a padded
// tile of its own, shorter remainders are packed, in run order, into the
// class's last tiles.  Output: orig[tile*64 + lane] = candidate index (-1 =
// padding), classes in order, and per class its tile count -- the same lane
// assignment as the host tiler, without taking the keys or the relaxed
// counts to the host.
//
// Every step is a map, an exclusive scan, or a scatter by scanned offsets;
// counts that size later steps stay on the device (kernels past them exit
// early), so the host waits once, for the per-class tile counts.
#include "fe_internal.h"

namespace fe {
namespace {

constexpr int TB = 256;           // threads per block
constexpr int TPT = 4;            // items per thread in the scans
constexpr int CHUNK = TB * TPT;   // items per scan block

__device__ __forceinline__ int key_dcls(const int *k, int m)
{
    int bound = 1;
    for (int j = 0; j < m - 1; ++j) {
        const int b = window_bound(k[3 * j + 1], k[3 * j + 2]);
        bound = b > bound ? b : bound;
    }
    return depth_class(bound);
}

// cls[i] = list-depth class of a kept candidate (0 for the relaxed pass),
// -1 for a pruned one
__global__ void k_tl_class(const int *__restrict__ key, int m, int64_t M,
                           const int *__restrict__ up, int theta, int exact, int *__restrict__ cls)
{
    const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
    if (i >= M) return;
    const int w = 3 * m - 2;
    const bool keep = !up || up[i] >= theta;
    cls[i] = !keep ? -1 : exact ? key_dcls(key + i * w, m) : 0;
}

// ---------------------------------------------------------------- scan
// Exclusive scan of v(i), i < n (n read from *np when np is set, else
// nfix): out[i] = sum of v(j), j < i; *total = sum of all.
struct ClassFlag {
    const int *cls;
    int c;
    __device__ int operator()(int64_t i) const { return cls[i] == c ? 1 : 0; }
};
struct Arr {
    const int *a;
    __device__ int operator()(int64_t i) const { return a[i]; }
};

__device__ __forceinline__ int64_t count_of(const int *np, int64_t nfix)
{
    return np ? (int64_t)*np : nfix;
}

// block sum of the values, and the block's exclusive prefix within LDS
__device__ __forceinline__ int block_excl(int v, int *sh, int &tot)
{
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == WAVE - 1) sh[wv] = x;
    __syncthreads();
    int base = 0, all = 0;
    for (int k = 0; k < TB / WAVE; ++k) {
        base += k < wv ? sh[k] : 0;
        all += sh[k];
    }
    __syncthreads();
    tot = all;
    return base + x - v;
}

template <class F>
__global__ void k_scan_up(F f, const int *np, int64_t nfix, int *__restrict__ bsum)
{
    __shared__ int sh[TB / WAVE];
    const int64_t n = count_of(np, nfix);
    const int64_t b0 = blockIdx.x * (int64_t)CHUNK;
    if (b0 >= n) {
        if (threadIdx.x == 0) bsum[blockIdx.x] = 0;
        return;
    }
    int s = 0;
    for (int k = 0; k < TPT; ++k) {
        const int64_t i = b0 + threadIdx.x * (int64_t)TPT + k;
        s += i < n ? f(i) : 0;
    }
    int tot;
    block_excl(s, sh, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// one block: exclusive scan of the nb block sums in place, total to *total
__global__ void k_scan_top(int *__restrict__ bsum, int64_t nb, int *__restrict__ total)
{
    __shared__ int sh[TB / WAVE];
    const int64_t per = (nb + TB - 1) / TB;
    const int64_t b = threadIdx.x * per, e = b + per < nb ? b + per : nb;
    int s = 0;
    for (int64_t i = b; i < e; ++i) s += bsum[i];
    int tot;
    int run = block_excl(s, sh, tot);
    for (int64_t i = b; i < e; ++i) {
        const int v = bsum[i];
        bsum[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) *total = tot;
}

template <class F>
__global__ void k_scan_down(F f, const int *np, int64_t nfix, const int *__restrict__ bsum,
                            int *__restrict__ out)
{
    __shared__ int sh[TB / WAVE];
    const int64_t n = count_of(np, nfix);
    const int64_t b0 = blockIdx.x * (int64_t)CHUNK;
    if (b0 >= n) return;
    int v[TPT], s = 0;
    for (int k = 0; k < TPT; ++k) {
        const int64_t i = b0 + threadIdx.x * (int64_t)TPT + k;
        v[k] = i < n ? f(i) : 0;
        s += v[k];
    }
    int tot;
    int run = bsum[blockIdx.x] + block_excl(s, sh, tot);
    for (int k = 0; k < TPT; ++k) {
        const int64_t i = b0 + threadIdx.x * (int64_t)TPT + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

template <class F>
void scan(F f, const int *np, int64_t nmax, int *out, int *bsum, int *total, hipStream_t s)
{
    const int64_t nb = (nmax + CHUNK - 1) / CHUNK;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TB), 0, s, bsum, (int64_t)0, total);
        return;
    }
    hipLaunchKernelGGL(k_scan_up<F>, dim3((unsigned)nb), dim3(TB), 0, s, f, np, nmax, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TB), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_down<F>, dim3((unsigned)nb), dim3(TB), 0, s, f, np, nmax, bsum,
                       out);
}

// ---------------------------------------------------------------- steps
// seg[c] = first position of class c in the partition, seg[NDCLS] = kept
__global__ void k_tl_seg(const int *__restrict__ ctot, int *__restrict__ seg)
{
    int acc = 0;
    for (int c = 0; c < NDCLS; ++c) {
        seg[c] = acc;
        acc += ctot[c];
    }
    seg[NDCLS] = acc;
}

// class c's candidates to part[] after those of classes 0..c-1
__global__ void k_tl_part(const int *__restrict__ cls, int64_t M, int c,
                          const int *__restrict__ pos, const int *__restrict__ ctot,
                          int *__restrict__ part)
{
    const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
    if (i >= M || cls[i] != c) return;
    int base = 0;
    for (int d = 0; d < c; ++d) base += ctot[d];
    part[base + pos[i]] = (int)i;
}

__device__ __forceinline__ int class_at(const int *seg, int j)
{
    int c = 0;
    for (int k = 1; k < NDCLS; ++k) c = j >= seg[k] ? k : c;
    return c;
}

// flag[j] = 1 where a run starts: a class's first position, or first m-1
// types differing from position j-1's
__global__ void k_tl_runflag(const int *__restrict__ part, const int *__restrict__ seg,
                             const int *__restrict__ key, int m, int *__restrict__ flag)
{
    const int64_t j = blockIdx.x * (int64_t)TB + threadIdx.x;
    const int S = seg[NDCLS];
    if (j >= S) return;
    bool start = j == 0;
    for (int c = 1; c < NDCLS; ++c) start |= j == seg[c];
    if (!start) {
        const int w = 3 * m - 2;
        const int *a = key + (int64_t)part[j - 1] * w, *b = key + (int64_t)part[j] * w;
        for (int k = 0; k < m - 1; ++k) start |= a[3 * k] != b[3 * k];
    }
    flag[j] = start ? 1 : 0;
}

__global__ void k_tl_runstart(const int *__restrict__ flag, const int *__restrict__ rx,
                              const int *__restrict__ seg, int *__restrict__ rs)
{
    const int64_t j = blockIdx.x * (int64_t)TB + threadIdx.x;
    if (j >= seg[NDCLS] || !flag[j]) return;
    rs[rx[j]] = (int)j;
}

// per run: tiles of its own (whole tiles, plus one padded when the remainder
// is at least half a tile) and lanes left for the class's packed tiles
__global__ void k_tl_runvals(const int *__restrict__ rs, const int *__restrict__ R,
                             const int *__restrict__ seg, int *__restrict__ rt,
                             int *__restrict__ rm)
{
    const int64_t r = blockIdx.x * (int64_t)TB + threadIdx.x;
    const int nr = *R;
    if (r >= nr) return;
    const int len = (r + 1 < nr ? rs[r + 1] : seg[NDCLS]) - rs[r];
    const int rem = len % WAVE;
    rt[r] = len / WAVE + (rem >= WAVE / 2 ? 1 : 0);
    rm[r] = rem >= WAVE / 2 ? 0 : rem;
}

// info[c]: tiles of class c; info[NDCLS + c]: its first tile; info[2*NDCLS +
// c]: its run tiles; info[3*NDCLS + c]: its first run; info[4*NDCLS + c]:
// candidates; info[5*NDCLS]: total tiles
__global__ void k_tl_groups(const int *__restrict__ seg, const int *__restrict__ rx,
                            const int *__restrict__ R, const int *__restrict__ toff,
                            const int *__restrict__ ttot, const int *__restrict__ moff,
                            const int *__restrict__ mtot, int *__restrict__ info)
{
    const int nr = *R;
    int base = 0;
    for (int c = 0; c < NDCLS; ++c) {
        const int n = seg[c + 1] - seg[c];
        int tiles = 0, rt = 0, fr = 0;
        if (n > 0) {
            fr = rx[seg[c]];
            int er = nr;  // first run of the next non-empty class
            for (int d = c + 1; d < NDCLS; ++d)
                if (seg[d + 1] > seg[d]) {
                    er = rx[seg[d]];
                    break;
                }
            const int t0 = toff[fr], t1 = er < nr ? toff[er] : *ttot;
            const int m0 = moff[fr], m1 = er < nr ? moff[er] : *mtot;
            rt = t1 - t0;
            tiles = rt + (m1 - m0 + WAVE - 1) / WAVE;
        }
        info[c] = tiles;
        info[NDCLS + c] = base;
        info[2 * NDCLS + c] = rt;
        info[3 * NDCLS + c] = fr;
        info[4 * NDCLS + c] = n;
        base += tiles;
    }
    info[5 * NDCLS] = base;
}

__global__ void k_tl_lanes(const int *__restrict__ part, const int *__restrict__ seg,
                           const int *__restrict__ flag, const int *__restrict__ rx,
                           const int *__restrict__ rs, const int *__restrict__ R,
                           const int *__restrict__ toff, const int *__restrict__ moff,
                           const int *__restrict__ info, int *__restrict__ orig)
{
    const int64_t j = blockIdx.x * (int64_t)TB + threadIdx.x;
    const int S = seg[NDCLS];
    if (j >= S) return;
    const int nr = *R;
    const int r = rx[j] + flag[j] - 1;
    const int len = (r + 1 < nr ? rs[r + 1] : S) - rs[r];
    const int k = (int)j - rs[r];
    const int full = len / WAVE, rem = len % WAVE;
    const int c = class_at(seg, (int)j);
    const int fr = info[3 * NDCLS + c], gbase = info[NDCLS + c];
    int tile, lane;
    if (k < full * WAVE || rem >= WAVE / 2) {
        const int q = toff[r] - toff[fr];
        tile = gbase + q + k / WAVE;
        lane = k % WAVE;
    } else {
        const int q = moff[r] - moff[fr] + (k - full * WAVE);
        tile = gbase + info[2 * NDCLS + c] + q / WAVE;
        lane = q % WAVE;
    }
    orig[(int64_t)tile * WAVE + lane] = part[j];
}

}  // namespace

int64_t tile_scratch_ints(int64_t M)
{
    // cls, pos, part, flag, rx, rs, rt, rm, toff, moff: M each; block sums
    // and small counters after them
    return 10 * M + (M + CHUNK - 1) / CHUNK + 64;
}

void launch_tile_plan(const int *key, int m, int64_t M, const int *up, int theta, bool exact,
                      int *scratch, int *info, hipStream_t s)
{
    int *cls = scratch, *pos = cls + M, *part = pos + M, *flag = part + M, *rx = flag + M;
    int *rs = rx + M, *rt = rs + M, *rm = rt + M, *toff = rm + M, *moff = toff + M;
    int *bsum = moff + M;
    int *small = bsum + (M + CHUNK - 1) / CHUNK;
    int *ctot = small, *seg = ctot + NDCLS, *R = seg + NDCLS + 1, *ttot = R + 1,
        *mtot = ttot + 1;
    const unsigned gM = (unsigned)((M + TB - 1) / TB);
    if (gM) hipLaunchKernelGGL(k_tl_class, dim3(gM), dim3(TB), 0, s, key, m, M, up, theta,
                               exact ? 1 : 0, cls);
    const int ncls = exact ? NDCLS : 1;
    for (int c = 0; c < NDCLS; ++c) {
        if (c < ncls) {
            scan(ClassFlag{cls, c}, nullptr, M, pos, bsum, ctot + c, s);
            if (gM) hipLaunchKernelGGL(k_tl_part, dim3(gM), dim3(TB), 0, s, cls, M, c, pos, ctot,
                                       part);
        } else {
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TB), 0, s, bsum, (int64_t)0, ctot + c);
        }
    }
    hipLaunchKernelGGL(k_tl_seg, dim3(1), dim3(1), 0, s, ctot, seg);
    if (gM) hipLaunchKernelGGL(k_tl_runflag, dim3(gM), dim3(TB), 0, s, part, seg, key, m, flag);
    scan(Arr{flag}, seg + NDCLS, M, rx, bsum, R, s);
    if (gM) hipLaunchKernelGGL(k_tl_runstart, dim3(gM), dim3(TB), 0, s, flag, rx, seg, rs);
    if (gM) hipLaunchKernelGGL(k_tl_runvals, dim3(gM), dim3(TB), 0, s, rs, R, seg, rt, rm);
    scan(Arr{rt}, R, M, toff, bsum, ttot, s);
    scan(Arr{rm}, R, M, moff, bsum, mtot, s);
    hipLaunchKernelGGL(k_tl_groups, dim3(1), dim3(1), 0, s, seg, rx, R, toff, ttot, moff, mtot,
                       info);
}

void launch_tile_lanes(int64_t M, const int *scratch, const int *info, int *orig, hipStream_t s)
{
    const int *part = scratch + 2 * M, *flag = scratch + 3 * M, *rx = scratch + 4 * M;
    const int *rs = scratch + 5 * M, *toff = scratch + 8 * M, *moff = scratch + 9 * M;
    const int *small = scratch + 10 * M + (M + CHUNK - 1) / CHUNK;
    const int *seg = small + NDCLS, *R = seg + NDCLS + 1;
    const unsigned gM = (unsigned)((M + TB - 1) / TB);
    if (gM) hipLaunchKernelGGL(k_tl_lanes, dim3(gM), dim3(TB), 0, s, part, seg, flag, rx, rs, R,
                               toff, moff, info, orig);
}

// ---------------------------------------------------------------- join
// Level m+1 candidates from the frequent m-node episodes F (sorted keys, w
// ints each): alpha's candidates are alpha's first node and hop followed by
// each beta in F whose first m-1 nodes and hops equal alpha's last m-1
// (first[a]: the first such beta; off[a]..off[a+1]: alpha's output range).
namespace {
__global__ void k_join(const int *__restrict__ F, int w, const int64_t *__restrict__ first,
                       const int64_t *__restrict__ off, int64_t cnt, int64_t M,
                       int *__restrict__ out)
{
    const int64_t j = blockIdx.x * (int64_t)TB + threadIdx.x;
    if (j >= M) return;
    int64_t lo = 0, hi = cnt;  // last a with off[a] <= j
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= j) lo = mid;
        else hi = mid;
    }
    const int64_t a = lo, b = first[a] + (j - off[a]);
    const int wo = w + 3;
    int *o = out + j * wo;
    const int *al = F + a * w, *be = F + b * w;
    o[0] = al[0];
    o[1] = al[1];
    o[2] = al[2];
    for (int k = 0; k < w; ++k) o[3 + k] = be[k];
}

__global__ void k_gather_keys(const int *__restrict__ key, int w, const int *__restrict__ sel,
                              int nsel, int *__restrict__ out)
{
    const int64_t t = blockIdx.x * (int64_t)TB + threadIdx.x;
    if (t >= (int64_t)nsel * w) return;
    const int64_t i = t / w;
    const int k = (int)(t - i * w);
    out[t] = key[(int64_t)sel[i] * w + k];
}
// Keys of a sample of the level: every SAMPLE_STRIDE-th block of WAVE
// consecutive candidates (whole blocks keep runs of join siblings together).
__global__ void k_sample_keys(const int *__restrict__ key, int w, int64_t ns,
                              int *__restrict__ out)
{
    const int64_t t = blockIdx.x * (int64_t)TB + threadIdx.x;
    if (t >= ns * w) return;
    const int64_t i = t / w;
    const int k = (int)(t - i * w);
    const int64_t j = i / WAVE * WAVE * SAMPLE_STRIDE + i % WAVE;
    out[t] = key[j * w + k];
}
}  // namespace

int64_t sample_count(int64_t M)
{
    const int64_t span = (int64_t)WAVE * SAMPLE_STRIDE;
    const int64_t r = M % span;
    return M / span * WAVE + (r < WAVE ? r : WAVE);
}

void launch_sample_keys(const int *key, int w, int64_t M, int *out, hipStream_t s)
{
    const int64_t n = sample_count(M) * w;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sample_keys, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, s, key, w,
                       sample_count(M), out);
}

int64_t scan_scratch_ints(int64_t n) { return (n + CHUNK - 1) / CHUNK + 1; }

void launch_scan_excl(const int *in, int64_t n, int *out, int *scratch, hipStream_t s)
{
    scan(Arr{in}, nullptr, n, out, scratch + 1, scratch, s);
}

void launch_join(const int *F, int w, const int64_t *first, const int64_t *off, int64_t cnt,
                 int64_t M, int *out, hipStream_t s)
{
    if (M <= 0 || cnt <= 0) return;
    hipLaunchKernelGGL(k_join, dim3((unsigned)((M + TB - 1) / TB)), dim3(TB), 0, s, F, w, first,
                       off, cnt, M, out);
}

void launch_gather_keys(const int *key, int w, const int *sel, int nsel, int *out, hipStream_t s)
{
    const int64_t n = (int64_t)nsel * w;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_keys, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, s, key, w,
                       sel, nsel, out);
}

}  // namespace fe
