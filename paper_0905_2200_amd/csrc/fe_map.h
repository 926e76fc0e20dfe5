// fe_map.h -- the Map step: per-lane episode state machines over a stream
// segment (MapConcatenate, Sec. 5.2.2), for the relaxed counter
// (Algorithm 3, Sec. 5.3.1) and the exact counter (Algorithm 1, Sec. 5.1).
// Instantiated per episode size N in fe_map_n<N>.hip.
//
// Mapping (CDNA4, wave64): one lane = one candidate's machine; one wave = a
// tile of 64 candidates over one segment.  Every lane reads the same event,
// so events come through scalar loads in the constant address space (one
// SMEM fetch serves 64 machines) and machine state stays in VGPRs.
//
// Counting semantics: for each event, nodes are visited from N down to 1
// against the state before the event; a node-i match whose hop test passes
// against list i-1 pushes t into list i; at node N it is a completion:
// count, clear every list, skip the rest of the event.  Node 1 always
// pushes.  N = 1 counts every event of its type.
//  * Relaxed (Algorithm 3): list k keeps its latest timestamp, held as the
//    deadline s_k + hi_k; the hop test is t <= deadline (gap in [0, hi]).
//  * Exact (Algorithm 1): a list matters only through the set of ticks that
//    pass its hop test, the union over entries e of [e+lo+1, e+hi].  Each
//    list is held as that union: sorted disjoint integer windows; windows
//    that ended before t are dropped, touching windows merged.  Live
//    entries lie in [t-hi, t] and unmerged neighbours are more than hi-lo
//    apart, so at most hi/(hi-lo+1)+1 windows are live; D is that bound,
//    fixed per candidate group at compile time.
//
// Exact stitching of segments: after a completion the machine is empty,
// every occurrence spans at most W = sum(hi) ticks, and completions happen
// only at events of type E_(N).  On segment [L, R) the true machine
// therefore behaves like a fresh machine started right after max(r, lam-1)
// (r = last completion before L, lam = first index with tick >= t_L - W).
// The restart points ("slots") are lam-1 and each E_(N) event in [lam, L);
// the Map step runs one machine per slot and writes, per slot, the
// completions it counts in [L, R) and the slot it leaves the next segment
// in.  Concatenate composes those tables.
#pragma once

#include "fe_internal.h"

namespace fe {

typedef const __attribute__((address_space(4))) int *cptr;
static constexpr int EMPTY = 0x7fffffff;

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int N> struct Cand {
    int ty[N];
    int lo[N > 1 ? N - 1 : 1];
    int hi[N > 1 ? N - 1 : 1];
};

template <int N> __device__ __forceinline__ void load_cand(Cand<N> &c, const int *rec, int lane)
{
#pragma unroll
    for (int k = 0; k < N; ++k) c.ty[k] = rec[k * WAVE + lane];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        c.lo[k] = rec[(N + k) * WAVE + lane];
        c.hi[k] = rec[(2 * N - 1 + k) * WAVE + lane];
    }
}

template <int N> struct Relaxed {
    int dl[N > 1 ? N - 1 : 1];
    __device__ __forceinline__ void reset()
    {
#pragma unroll
        for (int k = 0; k < N - 1; ++k) dl[k] = -1;
    }
    __device__ __forceinline__ bool step(int e, int t, const Cand<N> &c, bool on, int *)
    {
        if constexpr (N == 1) {
            return on & (e == c.ty[0]);
        } else {
            const bool comp = on & (e == c.ty[N - 1]) & (t <= dl[N - 2]);
#pragma unroll
            for (int i = N - 2; i >= 1; --i) {
                const bool ok = on & (e == c.ty[i]) & (t <= dl[i - 1]);
                dl[i] = ok ? t + c.hi[i] : dl[i];
            }
            const bool m0 = on & (e == c.ty[0]);
            dl[0] = m0 ? t + c.hi[0] : dl[0];
            return comp;
        }
    }
};

template <int N, int D> struct Exact {
    int wa[N > 1 ? N - 1 : 1][D];
    int wb[N > 1 ? N - 1 : 1][D];
    __device__ __forceinline__ void reset()
    {
#pragma unroll
        for (int k = 0; k < N - 1; ++k)
#pragma unroll
            for (int d = 0; d < D; ++d) { wa[k][d] = EMPTY; wb[k][d] = EMPTY; }
    }
    __device__ __forceinline__ bool hit(int k, int t) const
    {
        bool h = false;
#pragma unroll
        for (int d = 0; d < D; ++d) h |= (wa[k][d] <= t) & (t <= wb[k][d]);
        return h;
    }
    __device__ __forceinline__ void push(int k, int t, int lo, int hi, int *status)
    {
        const int a = t + lo + 1, b = t + hi;
        int nd = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) nd += wb[k][d] < t ? 1 : 0;
        int na[D], nb[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            na[d] = EMPTY;
            nb[d] = EMPTY;
#pragma unroll
            for (int s = 0; s + d < D; ++s)
                if (s == nd) { na[d] = wa[k][d + s]; nb[d] = wb[k][d + s]; }
        }
        int lc = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) lc += nb[d] != EMPTY ? 1 : 0;
        bool merged = false;
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (d == lc - 1 && nb[d] >= a - 1) { nb[d] = b; merged = true; }
        if (!merged) {
            if (lc < D) {
#pragma unroll
                for (int d = 0; d < D; ++d)
                    if (d == lc) { na[d] = a; nb[d] = b; }
            } else {
                atomicOr(status, ST_INTERNAL);
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) { wa[k][d] = na[d]; wb[k][d] = nb[d]; }
    }
    __device__ __forceinline__ bool step(int e, int t, const Cand<N> &c, bool on, int *status)
    {
        if constexpr (N == 1) {
            return on & (e == c.ty[0]);
        } else {
            const bool comp = on & (e == c.ty[N - 1]) & hit(N - 2, t);
#pragma unroll
            for (int i = N - 2; i >= 1; --i)
                if (on & (e == c.ty[i]) & hit(i - 1, t)) push(i, t, c.lo[i], c.hi[i], status);
            if (on & (e == c.ty[0])) push(0, t, c.lo[0], c.hi[0], status);
            return comp;
        }
    }
};

template <int N, bool EXACT, int D> struct MachineOf { typedef Relaxed<N> type; };
template <int N, int D> struct MachineOf<N, true, D> { typedef Exact<N, D> type; };

// Stream [b, e) (wave-uniform bounds) through scalar loads, U events per
// fetch, calling f(id, tick, index) in stream order.
template <int U, class F>
__device__ __forceinline__ void for_events(cptr ids, cptr ticks, int b, int e, F &&f)
{
    int i = uniform(b);
    e = uniform(e);
    for (; i + U <= e; i += U) {
        int ev[U], tv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) { ev[k] = ids[i + k]; tv[k] = ticks[i + k]; }
#pragma unroll
        for (int k = 0; k < U; ++k) f(ev[k], tv[k], i + k);
    }
    for (; i < e; ++i) f(ids[i], ticks[i], i);
}

// One machine run with the Map step's bookkeeping.  GUARD: lanes start at
// their own index `start` (slot machines) and only lanes with `act` run.
template <int N, bool EXACT, int D, bool GUARD> struct Run {
    static constexpr int U = EXACT ? (D >= 4 || N >= 6 ? 2 : 4) : 8;
    typename MachineOf<N, EXACT, D>::type m;
    int cnt = 0;    // completions counted
    int lastx = 0;  // exit slot in the next segment implied by the last completion
    int nx = 0;     // E_(N) events seen at index >= lamn (exit numbering)
    int start = 0;
    bool act = true;
    int ks = 0, s0 = -1, s1 = -1, s2 = -1;  // look-back E_(N) positions (slots 1..3)

    __device__ __forceinline__ bool on(int idx) const
    {
        if constexpr (GUARD) return act & (idx >= start);
        else return true;
    }

    // Bulk of a segment: count every completion; no exit bookkeeping (only
    // called on indices below the next segment's look-back).
    __device__ void body(cptr ids, cptr ticks, int b, int e, const Cand<N> &c, int *status)
    {
        if (uniform(b) >= uniform(e)) return;
        for_events<U>(ids, ticks, b, e, [&](int ev, int t, int idx) {
            if (m.step(ev, t, c, on(idx), status)) {
                m.reset();
                ++cnt;
                lastx = 0;
            }
        });
    }

    // Edges of a segment (look-back and the next segment's look-back):
    // completions count only at idx >= L, an exit slot is numbered at
    // idx >= lamn, and with rec the E_(N) events before L are recorded.
    __device__ void edge(cptr ids, cptr ticks, int b, int e, int L, int lamn, bool rec,
                         const Cand<N> &c, int *status)
    {
        if (uniform(b) >= uniform(e)) return;
        for_events<U>(ids, ticks, b, e, [&](int ev, int t, int idx) {
            const bool o = on(idx);
            const bool comp = m.step(ev, t, c, o, status);
            const bool nx_on = idx >= lamn;
            if (comp) {
                m.reset();
                cnt += idx >= L ? 1 : 0;
                lastx = nx_on ? nx + 1 : 0;
            }
            const bool isN = o & (ev == c.ty[N - 1]);
            nx += (nx_on & isN) ? 1 : 0;
            if (rec & (idx < L) & isN) {
                s0 = ks == 0 ? idx : s0;
                s1 = ks == 1 ? idx : s1;
                s2 = ks == 2 ? idx : s2;
                ++ks;
            }
        });
    }
};

template <int N, bool EXACT, int D>
__global__ __launch_bounds__(WAVE *WPB) void k_map(const int *__restrict__ ids_,
                                                   const int *__restrict__ ticks_, MapGroup g)
{
    static_assert(KMAX == 4, "slot recording holds KMAX-1 = 3 positions");
    cptr ids = (cptr)ids_;
    cptr ticks = (cptr)ticks_;
    const int lane = __lane_id();
    const int w = uniform(blockIdx.x * WPB + (threadIdx.x >> 6));
    const int P = g.P, tiles = g.tiles;
    if (w >= tiles * P) return;
    const int p = w / tiles, tile = w - p * tiles;
    const int c = tile * WAVE + lane;
    const int o = g.orig[c];

    Cand<N> cd;
    load_cand<N>(cd, g.pk + (int64_t)tile * rec_ints(N), lane);

    Run<N, EXACT, D, false> r;
    r.m.reset();
    if (P == 1) {
        r.body(ids, ticks, 0, g.n, cd, g.status);
        if (o >= 0) g.out[o] = r.cnt;
        return;
    }

    const int n = g.n;
    const int L = (int)((int64_t)p * n / P);
    const int R = (int)((int64_t)(p + 1) * n / P);
    const int lam = uniform(g.lam[(int64_t)tile * (P + 1) + p]);
    const int lamn = uniform(g.lam[(int64_t)tile * (P + 1) + p + 1]);
    const int x = lamn < lam ? lam : (lamn > R ? R : lamn);
    const int xl = x > L ? x : L;
    int2 *tb = g.tbl + ((int64_t)p * tiles * WAVE + c) * KMAX;

    // slot 0: the last completion before L lies before lam
    r.edge(ids, ticks, lam, L, L, lamn, true, cd, g.status);
    r.body(ids, ticks, L, xl, cd, g.status);
    r.edge(ids, ticks, xl, R, L, lamn, false, cd, g.status);
    tb[0] = make_int2(r.cnt, r.lastx < KMAX ? r.lastx : KMAX - 1);

    const int ks = r.ks;
    const bool ovf = ks > KMAX - 1;
    if (ovf && o >= 0) g.flags[c] = 1;
    // recorded slots that lie before the next segment's look-back
    const int fk = (ks > 0 && r.s0 < lamn) + (ks > 1 && r.s1 < lamn) + (ks > 2 && r.s2 < lamn);

    // slot j: the last completion before L is the j-th E_(N) event in [lam, L)
    for (int j = 1; j < KMAX; ++j) {
        const bool act = !ovf && o >= 0 && ks >= j;
        if (__ballot(act) == 0) break;
        const int sig = j == 1 ? r.s0 : (j == 2 ? r.s1 : r.s2);
        Run<N, EXACT, D, true> q;
        q.m.reset();
        q.act = act;
        q.start = sig + 1;
        q.nx = j - fk > 0 ? j - fk : 0;
        q.lastx = sig >= lamn ? j - fk : 0;
        int b = act ? sig + 1 : 0x7fffffff;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const int ob = __shfl_xor(b, off);
            b = ob < b ? ob : b;
        }
        b = uniform(b);
        q.edge(ids, ticks, b, L, L, lamn, false, cd, g.status);
        const int bl = b > L ? b : L;
        q.body(ids, ticks, bl, xl > bl ? xl : bl, cd, g.status);
        q.edge(ids, ticks, xl > bl ? xl : bl, R, L, lamn, false, cd, g.status);
        if (act) tb[j] = make_int2(q.cnt, q.lastx < KMAX ? q.lastx : KMAX - 1);
    }
}

// Recount candidates flagged by the Map step (a look-back held more than
// KMAX-1 slots) with one machine over the whole stream.
template <int N, bool EXACT, int D>
__global__ __launch_bounds__(WAVE *WPB) void k_fixup(const int *__restrict__ ids_,
                                                     const int *__restrict__ ticks_, MapGroup g)
{
    cptr ids = (cptr)ids_;
    cptr ticks = (cptr)ticks_;
    const int lane = __lane_id();
    const int tile = uniform(blockIdx.x * WPB + (threadIdx.x >> 6));
    if (tile >= g.tiles) return;
    const int c = tile * WAVE + lane;
    const int o = g.orig[c];
    const bool f = o >= 0 && g.flags[c] != 0;
    if (__ballot(f) == 0) return;
    Cand<N> cd;
    load_cand<N>(cd, g.pk + (int64_t)tile * rec_ints(N), lane);
    Run<N, EXACT, D, true> r;
    r.m.reset();
    r.act = f;
    r.start = 0;
    r.body(ids, ticks, 0, g.n, cd, g.status);
    if (f) g.out[o] = r.cnt;
}

template <int N, bool EXACT, int D> void map_n(const MapGroup &g, hipStream_t s, bool fix)
{
    if (fix) {
        hipLaunchKernelGGL((k_fixup<N, EXACT, D>), dim3((unsigned)((g.tiles + WPB - 1) / WPB)),
                           dim3(WAVE * WPB), 0, s, g.ids, g.ticks, g);
    } else {
        const int64_t items = (int64_t)g.tiles * g.P;
        hipLaunchKernelGGL((k_map<N, EXACT, D>), dim3((unsigned)((items + WPB - 1) / WPB)),
                           dim3(WAVE * WPB), 0, s, g.ids, g.ticks, g);
    }
}

template <int N> void map_dispatch_n(bool exact, int dcls, const MapGroup &g, hipStream_t s,
                                     bool fix)
{
    if (!exact) return map_n<N, false, 1>(g, s, fix);
    switch (dcls) {
    case 0: return map_n<N, true, 1>(g, s, fix);
    case 1: return map_n<N, true, 2>(g, s, fix);
    case 2: return map_n<N, true, 4>(g, s, fix);
    default: return map_n<N, true, 8>(g, s, fix);
    }
}

}  // namespace fe
