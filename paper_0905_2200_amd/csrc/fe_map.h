// fe_map.h -- the Map step: per-lane episode state machines over a stream
// segment (MapConcatenate, Sec. 5.2.2), for the relaxed counter
// (Algorithm 3, Sec. 5.3.1) and the exact counter (Algorithm 1, Sec. 5.1).
// Instantiated per episode size N in fe_map_n<N>.hip.
//
// Mapping (CDNA4, wave64): one lane = one candidate's machine; one wave = a
// tile of 64 candidates over one segment; machine state stays in VGPRs.
// Candidates produced by the level-wise join arrive in tiles whose first
// N-1 node types are the same in every lane; such waves test those nodes
// with scalar compares and only the last node per lane.  Two ways of
// feeding events (chosen per launch):
//  * per-type dispatch (sparse, sparse_lane): 64 events per vector load,
//    one per lane, with a per-block LDS table from type hash to event
//    positions, so that a lane steps only the events of its own types;
//  * every event through every lane (body): events through scalar loads in
//    the constant address space, one SMEM fetch serving 64 machines.
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
//    list is held as that union: disjoint integer windows in push order,
//    touching windows merged, the D most recent kept (older ones ended
//    before t).  Live entries lie in [t-hi, t] and unmerged neighbours are
//    more than hi-lo apart, so at most hi/(hi-lo+1)+1 windows are live; D
//    is that bound, fixed per candidate group at compile time.
//
// Exact stitching of segments: after a completion the machine is empty,
// every occurrence spans at most W = sum(hi) ticks, and completions happen
// only at events of type E_(N).  On segment [L, R) the true machine
// therefore behaves like a fresh machine started right after max(r, lam-1)
// (r = last completion before L, lam = first index with tick >= t_L - W).
// The restart points ("slots") are lam-1 (slot 0) and the j-th E_(N) event
// in [lam, L) (slot j).  The Map step runs one machine per slot and writes,
// per slot, the completions it counts in [L, R) and the slot it leaves the
// next segment in; Concatenate composes those tables.  Two machines that
// complete at the same event are identical from then on, so a slot machine
// stops at its first completion shared with the slot-0 machine and takes
// the rest of the result from it.
#pragma once

#include "fe_internal.h"

#include <type_traits>

namespace fe {

typedef const __attribute__((address_space(4))) int *cptr;
static constexpr int EMPTY = 0x7fffffff;  // start of a window slot never used
static constexpr int GONE = -0x7fffffff - 1;  // end of an unused or cleared window slot
static constexpr int QREC = 4;  // slot-0 completions remembered for merging

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-type dispatch reads the stream 64 events per vector load through
// buffer resources, whose range check returns 0 past the end (the prefetch
// of the block after the last one), with the block offset in an SGPR.  A
// resource covers at most EV_CHUNK events, so byte offsets stay below 2^31.
static constexpr int EV_CHUNK = 1 << 28;
static constexpr int BUF_DW3 = 0x00020000;  // raw 32-bit buffer access (gfx9)
struct EvBuf {
    __amdgpu_buffer_rsrc_t ri, rt;
    __device__ __forceinline__ EvBuf(const int *ids, const int *ticks, int cb, int ce)
        : ri(__builtin_amdgcn_make_buffer_rsrc((void *)(ids + cb), 0, (ce - cb) * 4, BUF_DW3)),
          rt(__builtin_amdgcn_make_buffer_rsrc((void *)(ticks + cb), 0, (ce - cb) * 4, BUF_DW3))
    {
    }
    // event rel + lane of the chunk (0 past its end)
    __device__ __forceinline__ void load(int rel, int lane4, int &id, int &tk) const
    {
        id = __builtin_amdgcn_raw_buffer_load_b32(ri, lane4, rel * 4, 0);
        tk = __builtin_amdgcn_raw_buffer_load_b32(rt, lane4, rel * 4, 0);
    }
    // the same, at byte offset boff = 4 rel
    __device__ __forceinline__ void load_b(int boff, int lane4, int &id, int &tk) const
    {
        id = __builtin_amdgcn_raw_buffer_load_b32(ri, lane4, boff, 0);
        tk = __builtin_amdgcn_raw_buffer_load_b32(rt, lane4, boff, 0);
    }
};

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

// Types of nodes 0..N-2 shared by every valid lane (wave-uniform values),
// and a 64-bit filter with bit (type & 63) set for each of them: an event
// whose bit is clear matches none of those nodes.
template <int N> struct Prefix {
    int ty[N > 1 ? N - 1 : 1];
    unsigned long long mask;
    __device__ __forceinline__ bool maybe(int e) const { return (mask >> (e & 63)) & 1ull; }
};

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
    // Event whose type matches none of nodes 0..N-2: only the last node acts.
    __device__ __forceinline__ bool step_last(int e, int t, const Cand<N> &c) const
    {
        if constexpr (N == 1) return e == c.ty[0];
        else return (e == c.ty[N - 1]) & (t <= dl[N - 2]);
    }
    // Latest tick list k's test passes at (-1 when empty).
    __device__ __forceinline__ int end_of(int k) const { return dl[k]; }
    __device__ __forceinline__ void flush(int *) {}
    // Nodes 0..N-2 have wave-uniform types u.ty: scalar tests, rare updates.
    __device__ __forceinline__ bool step_u(int e, int t, const Cand<N> &c, const Prefix<N> &u,
                                           int *)
    {
        if constexpr (N == 1) {
            return e == c.ty[0];
        } else {
            const bool comp = (e == c.ty[N - 1]) & (t <= dl[N - 2]);
            if (__builtin_expect(u.maybe(e), 0)) {
#pragma unroll
                for (int i = N - 2; i >= 1; --i)
                    if (e == u.ty[i]) dl[i] = t <= dl[i - 1] ? t + c.hi[i] : dl[i];
                if (e == u.ty[0]) dl[0] = t + c.hi[0];
            }
            return comp;
        }
    }
    // Nodes 0..N-2 of a shared-prefix wave only (the last node's test is
    // taken elsewhere); lanes with on = false leave their lists as they are.
    // (lm, hm: unused; the relaxed hop test is as cheap as a bound test)
    __device__ __forceinline__ void push_u(int e, int t, const Cand<N> &c, const Prefix<N> &u,
                                           bool on, int *, int *, const int *)
    {
        if constexpr (N > 1) {
#pragma unroll
            for (int i = N - 2; i >= 1; --i)
                if (__builtin_expect(e == u.ty[i], 0))
                    dl[i] = (on & (t <= dl[i - 1])) ? t + c.hi[i] : dl[i];
            if (__builtin_expect(e == u.ty[0], 0)) dl[0] = on ? t + c.hi[0] : dl[0];
        }
    }
};

template <int N, int D> struct Exact {
    // List k holds its D most recent windows in push order, slot D-1 the
    // newest: every window of a list has the same length and starts no
    // earlier than the ones before it, so windows end in slot order and a
    // window's successors are live whenever it is.  An unused slot ends at
    // GONE, before every tick.
    int wa[N > 1 ? N - 1 : 1][D];
    int wb[N > 1 ? N - 1 : 1][D];
    __device__ __forceinline__ Exact()
    {
#pragma unroll
        for (int k = 0; k < N - 1; ++k)
#pragma unroll
            for (int d = 0; d < D; ++d) { wa[k][d] = EMPTY; wb[k][d] = GONE; }
    }
    // Empty lists: every window ends before any tick, so no hop test passes.
    __device__ __forceinline__ void reset()
    {
#pragma unroll
        for (int k = 0; k < N - 1; ++k)
#pragma unroll
            for (int d = 0; d < D; ++d) {
                wa[k][d] = EMPTY;
                wb[k][d] = GONE;
            }
    }
    // reset() for the lanes with p, without a branch
    __device__ __forceinline__ void reset_p(bool p)
    {
#pragma unroll
        for (int k = 0; k < N - 1; ++k)
#pragma unroll
            for (int d = 0; d < D; ++d) {
                wa[k][d] = p ? EMPTY : wa[k][d];
                wb[k][d] = p ? GONE : wb[k][d];
            }
    }
    // t in [wa, wb] as one unsigned compare per window: t - wa <= wb - wa
    // (mod 2^32).  Live windows have wa <= wb and ticks below 2^30; an unused
    // slot (EMPTY, GONE) gives wb - wa = 1 and t - wa >= 2^31.
    __device__ __forceinline__ bool hit(int k, int t) const
    {
        bool h = false;
#pragma unroll
        for (int d = 0; d < D; ++d)
            h |= (unsigned)t - (unsigned)wa[k][d] <= (unsigned)wb[k][d] - (unsigned)wa[k][d];
        return h;
    }
    // Latest tick a window of list k covers (GONE when the list is empty):
    // no later tick can pass that list's test.
    __device__ __forceinline__ int end_of(int k) const { return wb[k][D - 1]; }
    // Window (t+lo, t+hi] joins the newest window when it overlaps or abuts
    // it, else it becomes the newest and the oldest is shifted out; that one
    // must have ended before t (at most D live windows, by the depth class).
    __device__ __forceinline__ void push(int k, int t, int lo, int hi, int *status)
    {
        const int a = t + lo + 1, b = t + hi;
        const bool mrg = wb[k][D - 1] >= a - 1;
        if (!mrg & (wb[k][0] >= t)) atomicOr(status, ST_INTERNAL);
#pragma unroll
        for (int d = 0; d + 1 < D; ++d) {
            wa[k][d] = mrg ? wa[k][d] : wa[k][d + 1];
            wb[k][d] = mrg ? wb[k][d] : wb[k][d + 1];
        }
        wa[k][D - 1] = mrg ? wa[k][D - 1] : a;
        wb[k][D - 1] = b;
    }
    // push() for the lanes with p, without a branch: a live window shifted
    // out (an overflow of the depth class, never expected) is remembered in
    // ovf and reported by flush()
    // (an int, so that it stays in a VGPR rather than a lane mask merged at
    // every branch)
    int ovf = 0;
    __device__ __forceinline__ void push_p(int k, int t, int lo, int hi, bool p)
    {
        const int a = t + lo + 1, b = t + hi;
        const bool sh = p & (wb[k][D - 1] < a - 1);
        ovf |= (sh & (wb[k][0] >= t)) ? 1 : 0;
#pragma unroll
        for (int d = 0; d + 1 < D; ++d) {
            wa[k][d] = sh ? wa[k][d + 1] : wa[k][d];
            wb[k][d] = sh ? wb[k][d + 1] : wb[k][d];
        }
        wa[k][D - 1] = sh ? a : wa[k][D - 1];
        wb[k][D - 1] = p ? b : wb[k][D - 1];
    }
    __device__ __forceinline__ void flush(int *status)
    {
        if (__builtin_amdgcn_ballot_w64(ovf != 0) != 0 && __lane_id() == 0)
            atomicOr(status, ST_INTERNAL);
        ovf = 0;
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
    __device__ __forceinline__ bool step_last(int e, int t, const Cand<N> &c) const
    {
        if constexpr (N == 1) return e == c.ty[0];
        else return (e == c.ty[N - 1]) & hit(N - 2, t);
    }
    __device__ __forceinline__ bool step_u(int e, int t, const Cand<N> &c, const Prefix<N> &u,
                                           int *status)
    {
        if constexpr (N == 1) {
            return e == c.ty[0];
        } else {
            const bool comp = (e == c.ty[N - 1]) & hit(N - 2, t);
            if (__builtin_expect(u.maybe(e), 0)) {
#pragma unroll
                for (int i = N - 2; i >= 1; --i)
                    if (e == u.ty[i])
                        if (hit(i - 1, t)) push(i, t, c.lo[i], c.hi[i], status);
                if (e == u.ty[0]) push(0, t, c.lo[0], c.hi[0], status);
            }
            return comp;
        }
    }
    // Nodes 0..N-2 of a shared-prefix wave only (the last node's test is
    // taken elsewhere); lanes with on = false leave their lists as they are.
    // lm[k]: a wave-uniform bound on every lane's end_of(k); hm[k]: the
    // wave's largest hi of hop k.  A node whose list k-1 passes at no lane
    // (t > lm[k-1]) is skipped whole.
    __device__ __forceinline__ void push_u(int e, int t, const Cand<N> &c, const Prefix<N> &u,
                                           bool on, int *status, int *lm, const int *hm)
    {
        if constexpr (N > 1) {
#pragma unroll
            for (int i = N - 2; i >= 1; --i)
                if (__builtin_expect(e == u.ty[i], 0))
                    if (t <= lm[i - 1]) {
                        lm[i] = t + hm[i];
                        push_p(i, t, c.lo[i], c.hi[i], on & hit(i - 1, t));
                    }
            if (__builtin_expect(e == u.ty[0], 0)) {
                lm[0] = t + hm[0];
                push_p(0, t, c.lo[0], c.hi[0], on);
            }
        }
    }
};

template <int N, bool EXACT, int D> struct MachineOf { typedef Relaxed<N> type; };
template <int N, int D> struct MachineOf<N, true, D> { typedef Exact<N, D> type; };

template <int N, bool EXACT, int D> struct Unroll {
    static constexpr int U = EXACT ? (D >= 4 || N >= 6 ? 2 : 4) : 8;
};

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

// The slot-0 machine of a segment (or the only machine when P = 1).
template <int N, bool EXACT, int D> struct MainRun {
    static constexpr int U = Unroll<N, EXACT, D>::U;
    typename MachineOf<N, EXACT, D>::type m;
    int cnt = 0;    // completions counted (index >= L)
    int lastx = 0;  // exit slot in the next segment implied by the last completion
    int nx = 0;     // E_(N) events seen at index >= lamn (exit numbering)
    int ks = 0;     // E_(N) events in the look-back [lam, L)
    int q = 0;      // completions seen; the first QREC are kept for merging
    int ci[QREC], ck[QREC], ct[QREC];  // index, count after it, tick
    int lastc = -1; // index of the last completion counted (whole-stream runs)

    __device__ __forceinline__ void note(int idx, int t)
    {
#pragma unroll
        for (int k = 0; k < QREC; ++k) {
            ci[k] = q == k ? idx : ci[k];
            ck[k] = q == k ? cnt : ck[k];
            ct[k] = q == k ? t : ct[k];
        }
        ++q;
    }

    // Bulk of a segment (indices below the next look-back): count every
    // completion.  UNI: the tile shares the types of nodes 0..N-2.
    __device__ __forceinline__ void complete(bool comp, int idx, int t, bool note_it)
    {
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(comp) != 0, 0)) {
            if (comp) {
                m.reset();
                ++cnt;
                lastx = 0;
                lastc = idx;
                if (note_it) note(idx, t);
            }
        }
    }

    // Bulk of a segment (indices below the next look-back): count every
    // completion.  UNI: the tile shares the types of nodes 0..N-2; then,
    // given per-chunk type masks of the stream (bit (type & 63) of every
    // event in an aligned chunk of 8), a chunk whose mask misses every
    // shared type is processed with the last node alone.
    template <bool UNI, bool NOTE, bool CHUNK = !EXACT>
    __device__ void body(cptr ids, cptr ticks, const unsigned long long *cmask, int b, int e,
                         const Cand<N> &c, const Prefix<N> &u, int *status)
    {
        b = uniform(b);
        e = uniform(e);
        if (b >= e) return;
        auto general = [&](int ev, int t, int idx) {
            bool comp;
            if constexpr (UNI) comp = m.step_u(ev, t, c, u, status);
            else comp = m.step(ev, t, c, true, status);
            complete(comp, idx, t, NOTE);
        };
        // (inside the segmented kernel the exact machine keeps the per-event
        // path: splitting its loop in two there grows the register copies of
        // its state past the occupancy budget)
        if constexpr (UNI && CHUNK) {
            if (cmask) {
                int i = b;
                const int a8 = (b + 7) & ~7;
                for (; i < e && i < a8; ++i) general(ids[i], ticks[i], i);
                for (; i + 8 <= e; i += 8) {
                    int ev[8], tv[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) { ev[k] = ids[i + k]; tv[k] = ticks[i + k]; }
                    const unsigned long long cm =
                        ((const __attribute__((address_space(4))) unsigned long long *)cmask)[i >> 3];
                    if ((cm & u.mask) == 0) {
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            complete(m.step_last(ev[k], tv[k], c), i + k, tv[k], NOTE);
                    } else if constexpr (EXACT) {
                        // rare: events of the shared-prefix types; the exact
                        // machine reloads them in a rolled loop, which keeps its
                        // register count (and occupancy) at the clean path's
#pragma unroll 1
                        for (int k = i; k < i + 8; ++k) general(ids[k], ticks[k], k);
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) general(ev[k], tv[k], i + k);
                    }
                }
                for (; i < e; ++i) general(ids[i], ticks[i], i);
                return;
            }
        }
        for_events<U>(ids, ticks, b, e, general);
    }

    // Bulk of a segment for a shared-prefix wave by per-type dispatch (the
    // paper's CPU counter keeps, per event type, the machines waiting on it;
    // this is the wave form of that idea).  Events come in blocks of 64, one
    // per lane (vector loads), and each block is written to LDS with a table
    // of event-position bits per type hash.  "Prefix events" (type hash of a
    // shared node) are stepped by the whole wave in stream order; of the
    // others a lane visits only those of its own last type.
    //   Only prefix events of node N-2's type change list N-2, the one the
    // last node tests, and so split the block into spans ending at such an
    // event (or at the block end).  Within a span the first last-type event
    // of a lane that passes the test -- prefix events included, the span's
    // closing one too, as completions come before pushes -- completes and
    // empties the machine; only one can, as list N-2 then stays empty to the
    // span's end.  Then the span's prefix events push in order, except, in
    // that lane, those at or before its completion.  tm, evs: this wave's
    // 64-entry LDS scratch.
    // hx: every type id is below 64 (each instantiation has one hot loop)
    template <bool NOTE>
    __device__ void sparse(const int *ids, const int *ticks, int b, int e, const Cand<N> &c,
                           const Prefix<N> &u, unsigned long long *tm, int2 *evs, int *status,
                           bool hx)
    {
        if (hx) sparse_t<NOTE, true>(ids, ticks, b, e, c, u, tm, evs, status);
        else sparse_t<NOTE, false>(ids, ticks, b, e, c, u, tm, evs, status);
    }
    template <bool NOTE, bool HX>
    __device__ void sparse_t(const int *ids, const int *ticks, int b, int e, const Cand<N> &c,
                             const Prefix<N> &u, unsigned long long *tm, int2 *evs, int *status)
    {
        static_assert(N >= 2, "per-type dispatch needs a shared prefix");
        b = uniform(b);
        e = uniform(e);
        if (b >= e) return;
        const int lane = __lane_id();
        const int dty = c.ty[N - 1];
        const int dh = dty & 63;
        const int lane4 = lane * 4;
        // wave-uniform bounds: hm[k] the largest hi of hop k, lm[k] >= every
        // lane's end_of(k) (raised at each node k event that may push)
        int hm[N - 1], lm[N - 1];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            hm[k] = 0;
            lm[k] = 0;
            if constexpr (!EXACT) continue;
            int x = c.hi[k], y = m.end_of(k);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const int ox = __shfl_xor(x, off), oy = __shfl_xor(y, off);
                x = ox > x ? ox : x;
                y = oy > y ? oy : y;
            }
            hm[k] = uniform(x);
            lm[k] = uniform(y);
        }
        for (int cb = b; cb < e; cb += EV_CHUNK) {
        const int ce = e - cb > EV_CHUNK ? cb + EV_CHUNK : e;
        const EvBuf eb(ids, ticks, cb, ce);
        int nid, ntk;
        eb.load(0, lane4, nid, ntk);
        // (full blocks and the final partial one are separate copies of the
        // body, so that full blocks need no position mask)
        auto block = [&](auto full_tag, int i) {
            constexpr bool FULL = decltype(full_tag)::value;
            const int id = nid, tk = ntk;
            eb.load(i - cb + WAVE, lane4, nid, ntk);
            const int left = ce - i;
            const bool v = FULL || lane < left;
            // positions holding events of this block (a wave-uniform mask)
            const unsigned long long vm = FULL ? ~0ull : (1ull << left) - 1ull;
            const int h = id & 63;
            tm[lane] = 0;
            evs[lane] = make_int2(id, tk);
            if (v) atomicOr(&tm[h], 1ull << lane);
            unsigned long long ml = tm[dh];
            const int tk0 = __builtin_amdgcn_readfirstlane(tk);
            // Prefix events that can act, per node: a node-k event (k >= 1)
            // changes a machine only where list k-1 passes at its tick.  When
            // no lane's list k-1 passes a tick from the block's first on,
            // that takes a node k-1 event earlier in the block that acts, so
            // node k's events up to the first such one are dropped.  Node
            // N-2's events that can act close the spans.
            unsigned long long eff = __builtin_amdgcn_ballot_w64(h == (u.ty[0] & 63)) & vm;
            unsigned long long pm = eff;
#pragma unroll
            for (int k = 1; k < N - 1; ++k) {
                const unsigned long long pk = __builtin_amdgcn_ballot_w64(h == (u.ty[k] & 63)) & vm;
                const bool live = EXACT ? lm[k - 1] >= tk0
                                        : __builtin_amdgcn_ballot_w64(m.end_of(k - 1) >= tk0) != 0;
                // (eff ^ (eff - 1): positions up to eff's first; all if none)
                eff = live ? pk : (pk & ~(eff ^ (eff - 1ull)));
                pm |= eff;
            }
            unsigned long long remp = pm, remb = eff;
            for (;;) {
                // span: positions up to the lowest closing event (all if none)
                const unsigned long long rb1 = remb - 1ull;
                const unsigned long long upto = remb ? (remb ^ rb1) : ~0ull;
                // list N-2 is fixed within the span; a lane whose list passes
                // no tick from the block's first on cannot complete
                unsigned long long gp = 0;
                int lim = GONE;
                if (!EXACT || lm[N - 2] >= tk0) {
                    gp = ml & upto;
                    lim = m.end_of(N - 2);
                    if (lim < tk0) gp = 0;
                }
                ml &= ~upto;
                int cpos = -1, ct = 0;
                // (one wave-uniform test skips the search in spans where no
                // lane has a last-type event that could complete, most of them)
                if (__builtin_amdgcn_ballot_w64(gp != 0) != 0) {
                    if constexpr (HX) {
                        // type ids below 64: every position in gp holds the last type
                        if constexpr (EXACT) {
                            while (gp) {
                                const int pos = (int)__builtin_ctzll(gp);
                                const int t = evs[pos].y;
                                const bool pass = m.step_last(dty, t, c);
                                if (pass | (t >= lim)) {
                                    // (ticks do not decrease: past the last window
                                    // no later event passes)
                                    cpos = pass ? pos : -1;
                                    ct = t;
                                    break;
                                }
                                gp &= gp - 1ull;
                            }
                        } else if (gp) {
                            const int pos = (int)__builtin_ctzll(gp);
                            const int t = evs[pos].y;
                            if (m.step_last(dty, t, c)) {
                                cpos = pos;
                                ct = t;
                            }
                        }
                    } else if constexpr (EXACT) {
                        // a later last-type event may enter a window an earlier one missed
                        while (gp) {
                            const int pos = (int)__builtin_ctzll(gp);
                            const int2 et = evs[pos];
                            // (et.x differs from dty only on a type-hash collision)
                            if ((et.x == dty) & m.step_last(et.x, et.y, c)) {
                                cpos = pos;
                                ct = et.y;
                                break;
                            }
                            if (et.y > lim) break;
                            gp &= gp - 1ull;
                        }
                    } else if (gp) {
                        // relaxed: only the first last-type event can pass (a later
                        // tick cannot pass a test this one failed); the loop skips
                        // type-hash collisions only
                        int pos = (int)__builtin_ctzll(gp);
                        int2 et = evs[pos];
                        while (et.x != dty && (gp &= gp - 1ull)) {
                            pos = (int)__builtin_ctzll(gp);
                            et = evs[pos];
                        }
                        if ((et.x == dty) & m.step_last(et.x, et.y, c)) {
                            cpos = pos;
                            ct = et.y;
                        }
                    }
                    if (cpos >= 0) {
                        m.reset();
                        ++cnt;
                        lastx = 0;
                        lastc = i + cpos;
                        if (NOTE) note(i + cpos, ct);
                    }
                }
                unsigned long long pp = remp & upto;
                remp &= ~upto;
                while (pp) {
                    const int x = (int)__builtin_ctzll(pp);
                    pp &= pp - 1ull;
                    const int ev = __builtin_amdgcn_readlane(id, x);
                    const int t = __builtin_amdgcn_readlane(tk, x);
                    m.push_u(ev, t, c, u, x > cpos, status, lm, hm);
                }
                if (!remb) break;
                remb &= rb1;
            }
        };
        int i = cb;
        for (; i + WAVE <= ce; i += WAVE) block(std::true_type(), i);
        if (i < ce) block(std::false_type(), i);
        }
        m.flush(status);
    }

    // Per-type dispatch for a wave without a shared prefix: in each block of
    // 64 events a lane visits, in stream order, only the events whose type
    // hash is one of its own nodes' (the others leave its machine as it is).
    // take: the lane takes part (padding lanes visit nothing).
    template <bool NOTE>
    __device__ void sparse_lane(const int *ids, const int *ticks, int b, int e, const Cand<N> &c,
                                bool take, unsigned long long *tm, int2 *evs, int *status)
    {
        b = uniform(b);
        e = uniform(e);
        if (b >= e) return;
        const int lane = __lane_id();
        const int lane4 = lane * 4;
        for (int cb = b; cb < e; cb += EV_CHUNK) {
        const int ce = e - cb > EV_CHUNK ? cb + EV_CHUNK : e;
        const EvBuf eb(ids, ticks, cb, ce);
        int nid, ntk;
        eb.load(0, lane4, nid, ntk);
        for (int i = cb; i < ce; i += WAVE) {
            const int id = nid, tk = ntk;
            eb.load(i - cb + WAVE, lane4, nid, ntk);
            tm[lane] = 0;
            evs[lane] = make_int2(id, tk);
            if (lane < ce - i) atomicOr(&tm[id & 63], 1ull << lane);
            // A node-k event (k >= 1) changes the machine only if list k-1
            // passes at its tick.  When list k-1 passes no tick from the
            // block's first on, that takes a node k-1 event earlier in the
            // block that acts, so node k's events up to the first such one
            // are skipped (the last node's too: it only completes).
            const int tk0 = __builtin_amdgcn_readfirstlane(tk);
            unsigned long long eff = tm[c.ty[0] & 63];
            unsigned long long ml = eff;
#pragma unroll
            for (int q = 1; q < N; ++q) {
                const unsigned long long mq = tm[c.ty[q] & 63];
                // (eff ^ (eff - 1): positions up to eff's first; all if none)
                eff = m.end_of(q - 1) >= tk0 ? mq : (mq & ~(eff ^ (eff - 1ull)));
                ml |= eff;
            }
            if (!take) ml = 0;
            while (ml) {
                const int pos = (int)__builtin_ctzll(ml);
                ml &= ml - 1ull;
                const int2 et = evs[pos];
                if (m.step(et.x, et.y, c, true, status)) {
                    m.reset();
                    ++cnt;
                    lastx = 0;
                    lastc = i + pos;
                    if (NOTE) note(i + pos, et.y);
                }
            }
        }
        }
    }

    // Look-back and tail of a segment: completions count only at idx >= L,
    // exit slots are numbered at idx >= lamn, look-back E_(N) events are
    // counted into ks.
    __device__ void edge(cptr ids, cptr ticks, int b, int e, int L, int lamn, const Cand<N> &c,
                         int *status)
    {
        if (uniform(b) >= uniform(e)) return;
        for_events<U>(ids, ticks, b, e, [&](int ev, int t, int idx) {
            const bool comp = m.step(ev, t, c, true, status);
            const bool nx_on = idx >= lamn;
            if (comp) {
                m.reset();
                cnt += idx >= L ? 1 : 0;
                lastx = nx_on ? nx + 1 : 0;
                note(idx, t);
            }
            const bool isN = ev == c.ty[N - 1];
            nx += (nx_on & isN) ? 1 : 0;
            ks += ((idx < L) & isN) ? 1 : 0;
        });
    }
};

// Slot j >= 1: a fresh machine started right after the j-th E_(N) event of
// the look-back.  It stops as soon as it is known to behave like the slot-0
// machine from then on, and takes the rest of the result from that machine:
//  * at a completion shared with a remembered slot-0 completion (both are
//    empty afterwards), or
//  * at the first event more than W ticks after the later of the two
//    machines' last reset points (their last completion, or the slot's
//    start): every list entry in which they can differ came from a chain
//    that began at or before that reset and would need more than W ticks to
//    reach the event, so both make the same decisions from there on.  This
//    needs every slot-0 completion before the event to be remembered, and
//    the event to lie before the next segment's look-back, so that the exit
//    slot is decided by later (shared) completions only.
template <int N, bool EXACT, int D>
__device__ void slot_pass(cptr ids, cptr ticks, int lam, int L, int R, int lamn, int j,
                          bool act, const Cand<N> &c, const MainRun<N, EXACT, D> &mr,
                          int *status, int &out_cnt, int &out_x)
{
    constexpr int U = Unroll<N, EXACT, D>::U;
    typename MachineOf<N, EXACT, D>::type m;
    m.reset();
    int W = 0;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) W += c.hi[k];
    int cnt = 0, lastx = 0, nx = 0, seen = 0;
    int rt = 0;  // tick of this machine's last reset point
    bool started = false, live = act;
    int i = uniform(lam);
    const int e = uniform(R);
    auto take_rest = [&](int ckk) {
        cnt += mr.cnt - ckk;
        lastx = mr.lastx;
        live = false;
    };
    // horizon test before processing event idx (tick t)
    auto horizon = [&](int idx, int t) {
        if (!(live & started) || idx > lamn) return;
        int kk = -1;
#pragma unroll
        for (int k = 0; k < QREC; ++k) kk = (k < mr.q && mr.ci[k] < idx) ? k : kk;
        const bool known = mr.q <= QREC || mr.ci[QREC - 1] >= idx;
        int mt = rt, ckk = 0;
#pragma unroll
        for (int k = 0; k < QREC; ++k)
            if (k == kk) {
                mt = mr.ct[k] > rt ? mr.ct[k] : rt;
                ckk = mr.ck[k];
            }
        if (known && t > mt + W) take_rest(ckk);
    };
    auto f = [&](int ev, int t, int idx) {
        const bool isN = ev == c.ty[N - 1];
        const bool nx_on = idx >= lamn;
        const bool comp = m.step(ev, t, c, live & started, status);
        if (comp) {
            m.reset();
            cnt += idx >= L ? 1 : 0;
            lastx = nx_on ? nx + 1 : 0;
            rt = t;
            // merge with the slot-0 machine at a shared completion
            int hitk = -1;
#pragma unroll
            for (int k = 0; k < QREC; ++k) hitk = (k < mr.q && mr.ci[k] == idx) ? k : hitk;
            if (hitk >= 0) {
                int ckk = 0;
#pragma unroll
                for (int k = 0; k < QREC; ++k) ckk = k == hitk ? mr.ck[k] : ckk;
                take_rest(ckk);
            }
        }
        const bool starts = live & !started & isN & (idx < L) & (seen + 1 == j);
        if (starts) {
            started = true;
            lastx = nx_on ? nx + 1 : 0;
            rt = t;
        }
        seen += (isN & (idx < L)) ? 1 : 0;
        nx += (isN & nx_on) ? 1 : 0;
    };
    for (; i + U <= e; i += U) {
        if (__ballot(live) == 0) break;
        int ev[U], tv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) { ev[k] = ids[i + k]; tv[k] = ticks[i + k]; }
        horizon(i, tv[0]);
#pragma unroll
        for (int k = 0; k < U; ++k) f(ev[k], tv[k], i + k);
    }
    for (; i < e; ++i) {
        if (__ballot(live) == 0) break;
        const int t = ticks[i];
        horizon(i, t);
        f(ids[i], t, i);
    }
    out_cnt = cnt;
    out_x = lastx;
}

// true when every valid lane has the same types in nodes 0..N-2
template <int N>
__device__ __forceinline__ bool shared_prefix(const Cand<N> &c, bool valid, Prefix<N> &u)
{
    if constexpr (N == 1) {
        return false;
    } else {
        const unsigned long long vm = __ballot(valid);
        if (vm == 0) return false;
        const int first = __ffsll((long long)vm) - 1;
        bool same = true;
        u.mask = 0;
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            u.ty[k] = uniform(__shfl(c.ty[k], first));
            same &= __ballot(valid & (c.ty[k] != u.ty[k])) == 0;
            u.mask |= 1ull << (u.ty[k] & 63);
        }
        return same;
    }
}

// Hop intervals 0..N-3 shared by every valid lane (wave-uniform values).
template <int N> struct UHops {
    int lo[N > 2 ? N - 2 : 1];
    int hi[N > 2 ? N - 2 : 1];
};

template <int N>
__device__ __forceinline__ bool shared_hops(const Cand<N> &c, bool valid, UHops<N> &h)
{
    if constexpr (N < 3) {
        return false;
    } else {
        const unsigned long long vm = __ballot(valid);
        if (vm == 0) return false;
        const int first = __ffsll((long long)vm) - 1;
        bool same = true;
#pragma unroll
        for (int k = 0; k < N - 2; ++k) {
            h.lo[k] = uniform(__shfl(c.lo[k], first));
            h.hi[k] = uniform(__shfl(c.hi[k], first));
            same &= __ballot(valid & ((c.lo[k] != h.lo[k]) | (c.hi[k] != h.hi[k]))) == 0;
        }
        return same;
    }
}

// Exact whole-stream Map of a wave whose lanes share the types of nodes
// 0..N-2 and the hops 0..N-3 (the join siblings of one frequent episode:
// they differ only in the last node and hop).  Lists 0..N-3 then receive
// the same events in every lane, except that a lane's completion empties
// its lists; so they are kept once per wave.  Each entry (tick, s) carries
// s, the stream index at which the newest chain of hop-passing events
// behind it starts (node 0: the event's own index); a lane's list holds
// exactly the entries with s after its last completion (by induction over
// the nodes: a chain lies after the completion iff its first event does).
// Along a list s does not decrease (a later event's newest predecessor in
// range is no older), so whether a node-k event at t passes hop k-1 -- an
// entry of list k-1 in [t - hi, t - lo - 1] -- and with which s is decided
// by the newest entry at or before t - lo - 1 alone.
//   Per lane remain list N-2 as windows (its hop differs by lane), the last
// node's test, the count and the index of the last completion.  In a block
// of 64 events (one per lane), node by node (so that the block's earlier
// events are in place), each node-k event enters list k (node 0: always;
// node k >= 1: when it passes against list k-1).  The node N-2 events that
// pass are list N-2's entries: they close spans as in the per-type dispatch
// (sparse_t), and enter a lane's windows when their s is after its last
// completion.  A block where no lane's list N-2 passes a tick from the
// block's first on and no entry arrives is done after the list updates.
//   Lists 0..N-3 are rings of the 64 newest entries held across the lanes
// of three registers (lane q: slot q), oldest to newest from the next slot
// to write; an entry is kept as the first and last tick its hop test passes
// at (tick + lo + 1, tick + hi) with its s; a ring starts full of unused
// slots that pass from GONE to GONE (in every search's count, never at a
// tick).  Ticks do not decrease along a ring, so the entries that pass from
// a tick t on or earlier are its first c slots in that order (c: a
// ballot's popcount), and the newest of them passes at t iff its last
// passing tick is at least t.  Overwriting an entry that could still pass a
// later test (its last passing tick at or after the block's first tick)
// ends the method with false: the caller then counts the tile with the
// general dispatch.
template <int N, int D, bool HX>
__device__ bool sparse_u(const int *ids, const int *ticks, int n, const Cand<N> &c,
                         const Prefix<N> &u, const UHops<N> &uh, unsigned long long *tm,
                         int2 *evs, int2 *scr, int *status, int &cnt_out)
{
    static_assert(N >= 3, "lists 0..N-3 must exist");
    constexpr int NR = N - 2;
    const int lane = __lane_id();
    const int lane4 = lane * 4;
    const int dty = c.ty[N - 1];
    const int dh = dty & 63;
    Exact<2, D> w;  // list N-2
    w.reset();
    int cnt = 0, rr = -1;
    // rings, slot `lane`: the first and last tick the entry's hop test
    // passes at (tick + lo_k + 1, tick + hi_k) and its s
    // (a ring starts full of unused slots that pass from GONE and to GONE:
    // counted by every search, oldest in ring order, never passing at a tick)
    int rl[NR], rh[NR], rs[NR];
    int hd[NR], nh[NR];  // slots ever written + 64, newest entry's last passing tick
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        rl[k] = GONE;
        rh[k] = GONE;
        rs[k] = 0;
        hd[k] = WAVE;
        nh[k] = GONE;
    }
    // wave-uniform: hm the largest hi of hop N-2, lm >= every lane's end_of
    int hm = c.hi[N - 2];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(hm, off);
        hm = o > hm ? o : hm;
    }
    hm = uniform(hm);
    int lm = GONE;
    // set in the lane of a slot whose entry was overwritten while it could
    // still pass a later test (the results are then discarded; every index
    // stays within the rings)
    int ovr = 0;
    // s of the block's list N-2 entries, in the lanes of their events (read
    // only at positions entered in the same block)
    int sv = 0;
    for (int cb = 0; cb < n; cb += EV_CHUNK) {
        const int ce = n - cb > EV_CHUNK ? cb + EV_CHUNK : n;
        const EvBuf eb(ids, ticks, cb, ce);
        int ia, ta, ib, tb, ic, tc;  // this block and the next two, in flight
        eb.load(0, lane4, ia, ta);
        eb.load(WAVE, lane4, ib, tb);
        // (full blocks and the final partial one are separate copies; full
        // blocks rotate three register sets, so each block's loads are
        // issued two blocks ahead)
        auto block = [&](auto full_tag, int i, int boff, const int id, const int tk, int &nid,
                         int &ntk) {
            constexpr bool FULL = decltype(full_tag)::value;
            eb.load_b(boff, lane4, nid, ntk);
            const int tk0 = __builtin_amdgcn_readfirstlane(tk);
            const unsigned long long vm = FULL ? ~0ull : (1ull << (ce - i)) - 1ull;
            // node 0: every event enters list 0 with s = its index
            const bool is0 = FULL ? id == u.ty[0] : (id == u.ty[0]) & (lane < ce - i);
            const unsigned long long m0 = __builtin_amdgcn_ballot_w64(is0);
            if (m0) {
                const int q = hd[0];
                const int c0 = __popcll(m0);
                // the block's node-0 events in order to scr[0..c0), then to
                // ring slots q, q+1, ... (other lanes write scr[WAVE], unread)
                const int rank = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(m0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m0, 0u));
                scr[is0 ? rank : WAVE] = make_int2(tk, i + lane);
                __builtin_amdgcn_wave_barrier();
                // (slots r >= c0 read a stale entry and keep their own; the
                // empty asm keeps the read whole rather than predicated)
                const int r = (lane - q) & (WAVE - 1);
                const bool take = r < c0;
                unsigned long long e = __builtin_bit_cast(unsigned long long, scr[r]);
                asm volatile("" : "+v"(e));
                const int et = (int)(unsigned)e, es = (int)(unsigned)(e >> 32);
                ovr |= (take & (rh[0] >= tk0)) ? 1 : 0;
                rl[0] = take ? et + uh.lo[0] + 1 : rl[0];
                rh[0] = take ? et + uh.hi[0] : rh[0];
                rs[0] = take ? es : rs[0];
                hd[0] = q + c0;
                nh[0] = __builtin_amdgcn_readlane(tk, 63 - __clzll(m0)) + uh.hi[0];
            }
            unsigned long long remb = 0;
#pragma unroll
            for (int k = 1; k <= N - 2; ++k) {
                // (skipped when no entry of list k-1 can lie in range of the
                // block's events, most blocks)
                if (nh[k - 1] < tk0) continue;
                // (node-k events after the newest entry's last passing tick
                // cannot pass: every older entry's window ends earlier)
                unsigned long long pk = __builtin_amdgcn_ballot_w64(id == u.ty[k]) &
                                        __builtin_amdgcn_ballot_w64(tk <= nh[k - 1]);
                if (!FULL) pk &= vm;
                const int base = hd[k - 1] - 1;
                while (pk) {
                    const int x = (int)__builtin_ctzll(pk);
                    // (clear bit x of the wave-uniform mask in one scalar
                    // instruction; the compiler's own form takes three)
                    asm("s_bitset0_b64 %0, %1" : "+s"(pk) : "s"(x));
                    const int t = __builtin_amdgcn_readlane(tk, x);
                    // entries whose test passes from t on or earlier: the first
                    // popcount in ring order
                    const unsigned long long le = __builtin_amdgcn_ballot_w64(rl[k - 1] <= t);
                    if (le == 0) continue;
                    const int q = (base + __popcll(le)) & (WAVE - 1);
                    if (__builtin_amdgcn_readlane(rh[k - 1], q) < t) continue;
                    const int s = __builtin_amdgcn_readlane(rs[k - 1], q);
                    if (k < N - 2) {
                        const bool at = lane == (hd[k] & (WAVE - 1));
                        ovr |= (at & (rh[k] >= tk0)) ? 1 : 0;
                        rl[k] = at ? t + uh.lo[k] + 1 : rl[k];
                        rh[k] = at ? t + uh.hi[k] : rh[k];
                        rs[k] = at ? s : rs[k];
                        ++hd[k];
                        nh[k] = t + uh.hi[k];
                    } else {
                        remb |= 1ull << x;
                        sv = lane == x ? s : sv;
                    }
                }
            }
            // (one scalar test: remb, or a nonzero mask while some lane's list
            // passes a tick of the block: lm >= tk0 iff some lane's tick is at
            // most lm, as in a full block every tick is at least tk0; lanes past
            // the end of a partial block read tick 0, which at worst sends that
            // one block on to an empty search)
            if ((remb | __builtin_amdgcn_ballot_w64(tk <= lm)) == 0) return;
            // type table of the block for the last node's search
            tm[lane] = 0;
            evs[lane] = make_int2(id, tk);
            if (FULL || lane < ce - i) atomicOr(&tm[id & 63], 1ull << lane);
            unsigned long long ml = tm[dh];
            for (;;) {
                // span: positions up to the lowest entry of list N-2 (all if none)
                const unsigned long long rb1 = remb - 1ull;
                const unsigned long long upto = remb ? (remb ^ rb1) : ~0ull;
                unsigned long long gp = 0;
                int lim = GONE;
                if (lm >= tk0) {
                    gp = ml & upto;
                    lim = w.end_of(0);
                    if (lim < tk0) gp = 0;
                }
                ml &= ~upto;
                int cpos = -1;
                if (__builtin_amdgcn_ballot_w64(gp != 0) != 0) {
                    if constexpr (HX) {
                        while (gp) {
                            const int pos = (int)__builtin_ctzll(gp);
                            const int t = evs[pos].y;
                            const bool pass = w.hit(0, t);
                            if (pass | (t >= lim)) {
                                cpos = pass ? pos : -1;
                                break;
                            }
                            gp &= gp - 1ull;
                        }
                    } else {
                        while (gp) {
                            const int pos = (int)__builtin_ctzll(gp);
                            const int2 et = evs[pos];
                            if ((et.x == dty) & w.hit(0, et.y)) {
                                cpos = pos;
                                break;
                            }
                            if (et.y > lim) break;
                            gp &= gp - 1ull;
                        }
                    }
                }
                if (__builtin_amdgcn_ballot_w64(cpos >= 0) != 0) {
                    const bool done = cpos >= 0;
                    w.reset_p(done);
                    cnt += done ? 1 : 0;
                    rr = done ? i + cpos : rr;
                }
                if (!remb) break;
                const int x = (int)__builtin_ctzll(remb);
                const int t = __builtin_amdgcn_readlane(tk, x);
                const bool on = __builtin_amdgcn_readlane(sv, x) > rr;
                w.push_p(0, t, c.lo[N - 2], c.hi[N - 2], on);
                if (__builtin_amdgcn_ballot_w64(on) != 0) lm = t + hm;
                remb &= rb1;
            }
        };
        int i = cb, boff = 8 * WAVE;  // (boff: byte offset of the block after the next)
        for (; i + 3 * WAVE <= ce; i += 3 * WAVE, boff += 12 * WAVE) {
            block(std::true_type(), i, boff, ia, ta, ic, tc);
            block(std::true_type(), i + WAVE, boff + 4 * WAVE, ib, tb, ia, ta);
            block(std::true_type(), i + 2 * WAVE, boff + 8 * WAVE, ic, tc, ib, tb);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (i + WAVE <= ce) {
                block(std::true_type(), i, boff, ia, ta, ic, tc);
                i += WAVE;
                boff += 4 * WAVE;
                ia = ib;
                ta = tb;
                ib = ic;
                tb = tc;
            }
        }
        if (i < ce) block(std::false_type(), i, boff, ia, ta, ic, tc);
    }
    w.flush(status);
    cnt_out = cnt;
    return __builtin_amdgcn_ballot_w64(ovr != 0) == 0;
}

// Everything one work item (a tile of 64 candidates over segment p of P)
// needs; shared by the per-group launch (k_map) and the persistent batched
// launch (k_persist).
struct ItemArgs {
    cptr ids, ticks;
    int n;
    const int *rec;  // the tile's packed record
    int P, p;
    const int *lam;  // the tile's look-back starts lam[0..P] (P > 1)
    int2 *tb;        // this lane's KMAX slot entries for segment p (P > 1)
    int *flag;       // this lane's slot-overflow flag (P > 1)
    int *out;        // counts, indexed by the candidate's input index
    int *status;
    const unsigned long long *cmask;  // per aligned 8-event chunk type masks, or null
    const int *gids, *gticks;         // the same stream for vector loads
    bool hashx;                       // every type id is below 64
    unsigned long long *tm;           // this wave's LDS scratch (per-type dispatch)
    int2 *evs;
};

// Map step of one work item.  o: the lane's candidate index (-1 = padding);
// valid: the lane's candidate takes part (its result is written).
template <int N, bool EXACT, int D, bool SPARSE>
__device__ __forceinline__ void map_item(const ItemArgs &a, int o, bool valid)
{
    Cand<N> cd;
    load_cand<N>(cd, a.rec, __lane_id());
    Prefix<N> u;
    const bool uni = shared_prefix<N>(cd, valid, u);

    MainRun<N, EXACT, D> r;
    r.m.reset();
    // bulk [b, e) of the segment, NOTE: remember slot-0 completions
    auto bulk = [&](auto note_tag, int b, int e) {
        constexpr bool NOTE = decltype(note_tag)::value;
        if constexpr (SPARSE) {
            bool done = false;
            if constexpr (N >= 2) {
                if (uni) {
                    r.template sparse<NOTE>(a.gids, a.gticks, b, e, cd, u, a.tm, a.evs, a.status,
                                            a.hashx);
                    done = true;
                }
            }
            if (!done)
                r.template sparse_lane<NOTE>(a.gids, a.gticks, b, e, cd, valid, a.tm, a.evs,
                                             a.status);
        } else if (uni) {
            r.template body<true, NOTE>(a.ids, a.ticks, a.cmask, b, e, cd, u, a.status);
        } else {
            r.template body<false, NOTE>(a.ids, a.ticks, a.cmask, b, e, cd, u, a.status);
        }
    };
    if (a.P == 1) {
        bulk(std::false_type(), 0, a.n);
        if (valid) a.out[o] = r.cnt;
        return;
    }

    const int n = a.n, P = a.P, p = a.p;
    const int L = (int)((int64_t)p * n / P);
    const int R = (int)((int64_t)(p + 1) * n / P);
    const int lam = uniform(a.lam[p]);
    const int lamn = uniform(a.lam[p + 1]);
    const int x = lamn < lam ? lam : (lamn > R ? R : lamn);
    const int xl = x > L ? x : L;

    // slot 0: the last completion before L lies before lam
    for (int k = 0; k < QREC; ++k) { r.ci[k] = -1; r.ck[k] = 0; r.ct[k] = 0; }
    r.edge(a.ids, a.ticks, lam, L, L, lamn, cd, a.status);
    bulk(std::true_type(), L, xl);
    r.edge(a.ids, a.ticks, xl, R, L, lamn, cd, a.status);
    if (valid) a.tb[0] = make_int2(r.cnt, r.lastx < KMAX ? r.lastx : KMAX - 1);

    const int K = r.ks + 1;  // slots of this lane
    const bool ovf = K > KMAX;
    if (ovf && valid) *a.flag = 1;
    int kw = (ovf || !valid) ? 1 : K;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int ok = __shfl_xor(kw, off);
        kw = ok > kw ? ok : kw;
    }
    kw = uniform(kw);
    for (int j = 1; j < kw; ++j) {
        const bool act = !ovf && valid && j < K;
        int sc = 0, sx = 0;
        slot_pass<N, EXACT, D>(a.ids, a.ticks, lam, L, R, lamn, j, act, cd, r, a.status, sc, sx);
        if (act) a.tb[j] = make_int2(sc, sx < KMAX ? sx : KMAX - 1);
    }
}

template <int N, bool EXACT, int D, bool SPARSE>
__global__ __launch_bounds__(WAVE *WPB) void k_map(const int *__restrict__ ids_,
                                                   const int *__restrict__ ticks_, MapGroup g)
{
    const int lane = __lane_id();
    const int w = uniform(blockIdx.x * WPB + (threadIdx.x >> 6));
    const int P = g.P, tiles = g.tiles;
    if (w >= tiles * P) return;
    const int p = w / tiles, tile = w - p * tiles;
    const int c = tile * WAVE + lane;
    const int o = g.orig[c];
    ItemArgs a;
    a.ids = (cptr)ids_;
    a.ticks = (cptr)ticks_;
    a.n = g.n;
    a.rec = g.pk + (int64_t)tile * rec_ints(N);
    a.P = P;
    a.p = p;
    a.lam = P > 1 ? g.lam + (int64_t)tile * (P + 1) : nullptr;
    a.tb = P > 1 ? g.tbl + ((int64_t)p * tiles * WAVE + c) * KMAX : nullptr;
    a.flag = P > 1 ? g.flags + c : nullptr;
    a.out = g.out;
    a.status = g.status;
    a.cmask = g.cmask;
    __shared__ unsigned long long s_tm[WPB][WAVE];
    __shared__ int2 s_ev[WPB][WAVE];
    a.gids = ids_;
    a.gticks = ticks_;
    a.tm = s_tm[threadIdx.x >> 6];
    a.evs = s_ev[threadIdx.x >> 6];
    a.hashx = g.hashx != 0;
    map_item<N, EXACT, D, SPARSE>(a, o, o >= 0);
}

// Whole-stream Map (P = 1, one machine per lane, no segment bookkeeping):
// the launch used when the tiles alone fill the GPU.  SPARSE: per-type
// dispatch (shared-prefix waves by gaps between prefix events, the others
// lane by lane); otherwise every event goes through every lane, shared-prefix
// waves skipping the 8-event chunks that hold no shared type.
template <int N, bool EXACT, int D, bool SPARSE>
__global__ __launch_bounds__(WAVE *WPB) void k_map1(const int *__restrict__ ids_,
                                                    const int *__restrict__ ticks_, MapGroup g)
{
    const int lane = __lane_id();
    const int tile = uniform(blockIdx.x * WPB + (threadIdx.x >> 6));
    if (tile >= g.tiles) return;
    const int o = g.orig[tile * WAVE + lane];
    Cand<N> cd;
    load_cand<N>(cd, g.pk + (int64_t)tile * rec_ints(N), lane);
    Prefix<N> u;
    const bool uni = shared_prefix<N>(cd, o >= 0, u);
    MainRun<N, EXACT, D> r;
    r.m.reset();
    if constexpr (SPARSE) {
        __shared__ unsigned long long s_tm[WPB][WAVE];
        __shared__ int2 s_ev[WPB][WAVE];
        const int wv = threadIdx.x >> 6;
        bool done = false;
        if constexpr (EXACT && N >= 3) {
            __shared__ int2 s_scr[WPB][WAVE + 1];
            UHops<N> uh;
            if (uni && g.shlists && shared_hops<N>(cd, o >= 0, uh)) {
                if (g.hashx)
                    done = sparse_u<N, D, true>(ids_, ticks_, g.n, cd, u, uh, s_tm[wv], s_ev[wv],
                                                s_scr[wv], g.status, r.cnt);
                else
                    done = sparse_u<N, D, false>(ids_, ticks_, g.n, cd, u, uh, s_tm[wv],
                                                 s_ev[wv], s_scr[wv], g.status, r.cnt);
                if (!done) r.cnt = 0;
            }
        }
        if constexpr (N >= 2) {
            if (uni && !done) {
                r.template sparse<false>(ids_, ticks_, 0, g.n, cd, u, s_tm[wv], s_ev[wv],
                                         g.status, g.hashx != 0);
                done = true;
            }
        }
        if (!done)
            r.template sparse_lane<false>(ids_, ticks_, 0, g.n, cd, o >= 0, s_tm[wv], s_ev[wv],
                                          g.status);
    } else {
        if (uni)
            r.template body<true, false, true>((cptr)ids_, (cptr)ticks_, g.cmask, 0, g.n, cd, u,
                                               g.status);
        else
            r.template body<false, false>((cptr)ids_, (cptr)ticks_, g.cmask, 0, g.n, cd, u,
                                          g.status);
    }
    if (o >= 0) g.out[o] = r.cnt;
}

// Incremental whole-stream Map: events [0, from) were counted by earlier
// calls, which left each candidate's count and last completion index r in
// count_io / last_io.  After a completion the machine is empty, and no
// occurrence spans more than W = sum(hi) ticks, so from `from` on the true
// machine behaves like a fresh one started after max(r, lam-1), lam being the
// first index with tick >= t_from - W; nor can that fresh machine complete
// before `from`.  Each lane runs such a machine from its own start (wave
// head: per-lane gate; then the shared bulk) and adds what it counts.
template <int N, bool EXACT, int D, bool SPARSE>
__global__ __launch_bounds__(WAVE *WPB) void k_resume(const int *__restrict__ ids_,
                                                      const int *__restrict__ ticks_, MapGroup g,
                                                      int from, int *count_io, int *last_io)
{
    const int lane = __lane_id();
    const int tile = uniform(blockIdx.x * WPB + (threadIdx.x >> 6));
    if (tile >= g.tiles) return;
    const int n = g.n;
    const int o = g.orig[tile * WAVE + lane];
    const bool valid = o >= 0;
    Cand<N> cd;
    load_cand<N>(cd, g.pk + (int64_t)tile * rec_ints(N), lane);
    Prefix<N> u;
    const bool uni = shared_prefix<N>(cd, valid, u);
    int st = n;  // this lane's first event
    int prev = -1;
    if (valid) {
        int W = 0;
#pragma unroll
        for (int k = 0; k < N - 1; ++k) W += cd.hi[k];
        const int x = ticks_[from] - W;
        int a = 0, b = from;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (ticks_[mid] < x) a = mid + 1;
            else b = mid;
        }
        prev = last_io[o];
        const int r1 = prev + 1 < 0 ? 0 : (prev + 1 > from ? from : prev + 1);
        st = r1 > a ? r1 : a;
    }
    int smin = st, smax = valid ? st : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int x1 = __shfl_xor(smin, off), x2 = __shfl_xor(smax, off);
        smin = x1 < smin ? x1 : smin;
        smax = x2 > smax ? x2 : smax;
    }
    smin = uniform(smin);
    smax = uniform(smax);
    if (smin >= n) return;
    MainRun<N, EXACT, D> r;
    r.m.reset();
    for_events<Unroll<N, EXACT, D>::U>((cptr)ids_, (cptr)ticks_, smin, smax,
                                       [&](int ev, int t, int idx) {
                                           if (r.m.step(ev, t, cd, valid & (idx >= st), g.status)) {
                                               r.m.reset();
                                               ++r.cnt;
                                               r.lastc = idx;
                                           }
                                       });
    if constexpr (SPARSE) {
        __shared__ unsigned long long s_tm[WPB][WAVE];
        __shared__ int2 s_ev[WPB][WAVE];
        const int wv = threadIdx.x >> 6;
        bool done = false;
        if constexpr (N >= 2) {
            if (uni) {
                r.template sparse<false>(ids_, ticks_, smax, n, cd, u, s_tm[wv], s_ev[wv],
                                         g.status, g.hashx != 0);
                done = true;
            }
        }
        if (!done)
            r.template sparse_lane<false>(ids_, ticks_, smax, n, cd, valid, s_tm[wv], s_ev[wv],
                                          g.status);
    } else {
        if (uni)
            r.template body<true, false>((cptr)ids_, (cptr)ticks_, nullptr, smax, n, cd, u,
                                         g.status);
        else
            r.template body<false, false>((cptr)ids_, (cptr)ticks_, nullptr, smax, n, cd, u,
                                          g.status);
    }
    if (valid) {
        count_io[o] += r.cnt;
        last_io[o] = r.lastc >= 0 ? r.lastc : prev;
    }
}

// Persistent batched Map: a grid sized to the machine pops (tile, segment)
// items of many recordings from a queue (heaviest first) until it is empty.
// In the exact pass only candidates that survived the relaxed pass count;
// the others get -1.
// (blocks of b.wpb waves, up to PERSIST_WPB_MAX; each wave's 1 KiB of
// dispatch scratch in dynamic LDS)
template <int N, bool EXACT, int D, bool SPARSE>
__global__ __launch_bounds__(WAVE *PERSIST_WPB_MAX) void k_persist(BatchDev b)
{
    extern __shared__ unsigned long long s_pdyn[];
    unsigned long long *s_tm = s_pdyn + (threadIdx.x >> 6) * 2 * WAVE;
    int2 *s_ev = (int2 *)(s_tm + WAVE);
    const int lane = __lane_id();
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(b.qctr, 1);
        it = uniform(__shfl(it, 0));
        if (it >= b.nitems) break;
        const int2 tp = b.items[it];
        const int tile = uniform(tp.x), p = uniform(tp.y);
        const TileDesc td = b.tiles[tile];
        const BJob jb = b.jobs[uniform(td.job)];
        const int c = tile * WAVE + lane;
        const int o = b.orig[(int64_t)uniform(td.otile) * WAVE + lane];
        int *out = EXACT ? jb.exact : jb.upper;
        bool valid = o >= 0;
        if (EXACT) valid = valid && jb.upper[o] >= jb.theta;
        const int P = uniform(td.P);
        if (EXACT && P == 1 && o >= 0 && !valid) out[o] = -1;
        if (__ballot(valid) == 0) continue;
        ItemArgs a;
        a.ids = (cptr)jb.ids;
        a.ticks = (cptr)jb.ticks;
        a.n = jb.n;
        a.rec = b.pk + td.rec;
        a.P = P;
        a.p = p;
        a.lam = b.lam + td.lam;
        a.tb = b.tbl + td.tbl + ((int64_t)p * WAVE + lane) * KMAX;
        a.flag = b.flags + c;
        a.out = out;
        a.status = b.status;
        a.cmask = nullptr;
        a.gids = jb.ids;
        a.gticks = jb.ticks;
        a.tm = s_tm;
        a.evs = s_ev;
        a.hashx = false;
        map_item<N, EXACT, D, SPARSE>(a, o, valid);
    }
}

// Recount candidates flagged by the Map step (a look-back held more than
// KMAX-1 restart slots) with one machine over the whole stream.
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
    typename MachineOf<N, EXACT, D>::type m;
    m.reset();
    int cnt = 0;
    for_events<Unroll<N, EXACT, D>::U>(ids, ticks, 0, g.n, [&](int ev, int t, int) {
        if (m.step(ev, t, cd, f, g.status)) {
            m.reset();
            ++cnt;
        }
    });
    if (f) g.out[o] = cnt;
}

// Batched recount of flagged candidates: one wave per listed tile.
template <int N, bool EXACT, int D>
__global__ __launch_bounds__(WAVE *WPB) void k_persist_fixup(BatchDev b, const int *ctiles,
                                                             int nct)
{
    const int lane = __lane_id();
    const int w = uniform(blockIdx.x * WPB + (threadIdx.x >> 6));
    if (w >= nct) return;
    const int tile = uniform(ctiles[w]);
    const TileDesc td = b.tiles[tile];
    const BJob jb = b.jobs[uniform(td.job)];
    const int c = tile * WAVE + lane;
    const int o = b.orig[(int64_t)uniform(td.otile) * WAVE + lane];
    bool f = o >= 0 && b.flags[c] != 0;
    if (EXACT) f = f && jb.upper[o] >= jb.theta;
    if (__ballot(f) == 0) return;
    Cand<N> cd;
    load_cand<N>(cd, b.pk + td.rec, lane);
    typename MachineOf<N, EXACT, D>::type m;
    m.reset();
    int cnt = 0;
    for_events<Unroll<N, EXACT, D>::U>((cptr)jb.ids, (cptr)jb.ticks, 0, jb.n,
                                       [&](int ev, int t, int) {
                                           if (m.step(ev, t, cd, f, b.status)) {
                                               m.reset();
                                               ++cnt;
                                           }
                                       });
    if (f) (EXACT ? jb.exact : jb.upper)[o] = cnt;
}

// Exact lists of the deep class (a hop with more than 8 live windows, e.g. a
// narrow interval far from 0 such as (190, 200] ticks).  The same windows as
// Exact<N, D> -- the union of [e+lo+1, e+hi] over the list's entries e, in
// push order, touching windows merged -- kept as a ring of `cap` windows per
// list in device memory, with the oldest kept window and the newest end in
// registers.  Windows that ended before the current tick are dropped from
// the front (ticks never decrease, so they can pass no later test); a hop
// test then only looks at the front window: live windows are disjoint and
// ordered, so if the tick is before the front one it is before all.  Live
// windows of list k end at or after t, so their last entries lie in
// [t-hi, t]: there are at most hi/(hi-lo+1)+1 of them and at most as many as
// events in that range, which sizes cap (overflow sets ST_INTERNAL).
template <int N> struct ExactDeep {
    static constexpr int L = N > 1 ? N - 1 : 1;
    int2 *w;       // this lane's rings: list k at w[k*cap ...]
    unsigned cap;
    unsigned head[L], cnt[L];
    int fa[L], fb[L];  // front window
    int nb[L];         // end of the newest window
    __device__ __forceinline__ void bind(int2 *ring, int c)
    {
        w = ring;
        cap = (unsigned)c;
    }
    __device__ __forceinline__ void reset()
    {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            head[k] = 0;
            cnt[k] = 0;
            fa[k] = EMPTY;
            fb[k] = GONE;
            nb[k] = GONE;
        }
    }
    __device__ __forceinline__ int end_of(int k) const { return nb[k]; }
    __device__ __forceinline__ void drop_dead(int k, int t)
    {
        while (cnt[k] != 0 && fb[k] < t) {
            head[k] = head[k] + 1 == cap ? 0 : head[k] + 1;
            if (--cnt[k] != 0) {
                const int2 v = w[(int64_t)k * cap + head[k]];
                fa[k] = v.x;
                fb[k] = v.y;
            } else {
                fa[k] = EMPTY;
                fb[k] = GONE;
                nb[k] = GONE;
            }
        }
    }
    __device__ __forceinline__ bool hit(int k, int t)
    {
        drop_dead(k, t);
        return cnt[k] != 0 && t >= fa[k];
    }
    __device__ __forceinline__ void push(int k, int t, int lo, int hi, int *status)
    {
        const int a = t + lo + 1, b = t + hi;
        drop_dead(k, t);
        if (cnt[k] != 0 && nb[k] >= a - 1) {
            // overlaps or abuts the newest window: extend it
            unsigned tail = head[k] + cnt[k] - 1;
            if (tail >= cap) tail -= cap;
            w[(int64_t)k * cap + tail].y = b;
            nb[k] = b;
            if (cnt[k] == 1) fb[k] = b;
            return;
        }
        if (cnt[k] == cap) {
            atomicOr(status, ST_INTERNAL);
            return;
        }
        unsigned tail = head[k] + cnt[k];
        if (tail >= cap) tail -= cap;
        w[(int64_t)k * cap + tail] = make_int2(a, b);
        if (cnt[k]++ == 0) {
            fa[k] = a;
            fb[k] = b;
        }
        nb[k] = b;
    }
    // Node loop of Algorithm 1 for one event (tested against the state
    // before the event, nodes N..1); true = completion at node N.
    __device__ __forceinline__ bool step(int e, int t, const Cand<N> &c, int *status)
    {
        if constexpr (N == 1) {
            return e == c.ty[0];
        } else {
            bool comp = false;
            if (e == c.ty[N - 1]) comp = hit(N - 2, t);
            if (comp) return true;  // the lists are cleared anyway
#pragma unroll
            for (int i = N - 2; i >= 1; --i)
                if (e == c.ty[i])
                    if (hit(i - 1, t)) push(i, t, c.lo[i], c.hi[i], status);
            if (e == c.ty[0]) push(0, t, c.lo[0], c.hi[0], status);
            return false;
        }
    }
};

// Whole-stream exact count of one chunk of a deep-class group: one wave per
// tile, lanes outside [g0, g1) idle.  Per-type dispatch lane by lane: in each
// block of 64 events a lane steps only the events whose type hash is one of
// its nodes' (the others leave its machine unchanged).  In the incremental
// form each lane starts after max(last completion, lam - 1) as in k_resume.
template <int N>
__global__ __launch_bounds__(WAVE *WPB) void k_deep(DeepArgs a)
{
    __shared__ unsigned long long s_tm[WPB][WAVE];
    __shared__ int2 s_ev[WPB][WAVE];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const int64_t tile = a.g0 / WAVE + uniform(blockIdx.x * WPB + wv);
    if (tile * WAVE >= a.g1) return;
    const int64_t gl = tile * WAVE + lane;
    const int o = a.orig[gl];
    bool on = o >= 0 && gl >= a.g0 && gl < a.g1;
    if (on && a.upper && a.upper[o] < a.theta) {
        a.out[o] = -1;
        on = false;
    }
    Cand<N> cd;
    load_cand<N>(cd, a.pk + tile * rec_ints(N), lane);
    ExactDeep<N> m;
    m.bind(a.ring + (on ? (gl - a.g0) * (int64_t)(N > 1 ? N - 1 : 1) * a.cap : 0), a.cap);
    m.reset();
    const int n = a.n;
    int st = on ? 0 : n;  // this lane's first event
    int prev = -1;
    if (on && a.count_io) {
        int W = 0;
#pragma unroll
        for (int k = 0; k < N - 1; ++k) W += cd.hi[k];
        st = n;
        if (a.from < n) {
            const int x = a.ticks[a.from] - W;
            int lo = 0, hi = a.from;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (a.ticks[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            prev = a.last_io[o];
            const int r1 = prev + 1 < 0 ? 0 : (prev + 1 > a.from ? a.from : prev + 1);
            st = r1 > lo ? r1 : lo;
        }
    }
    int smin = st;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int x = __shfl_xor(smin, off);
        smin = x < smin ? x : smin;
    }
    smin = uniform(smin);
    int cnt = 0, lastc = -1;
    unsigned long long *tm = s_tm[wv];
    int2 *evs = s_ev[wv];
    const int lane4 = lane * 4;
    for (int cb = smin; cb < n; cb += EV_CHUNK) {
        const int ce = n - cb > EV_CHUNK ? cb + EV_CHUNK : n;
        const EvBuf eb(a.ids, a.ticks, cb, ce);
        int nid, ntk;
        eb.load(0, lane4, nid, ntk);
        for (int i = cb; i < ce; i += WAVE) {
            const int id = nid, tk = ntk;
            eb.load(i - cb + WAVE, lane4, nid, ntk);
            tm[lane] = 0;
            evs[lane] = make_int2(id, tk);
            if (lane < ce - i) atomicOr(&tm[id & 63], 1ull << lane);
            unsigned long long ml = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) ml |= tm[cd.ty[q] & 63];
            // positions before this lane's start
            if (st > i) ml = st - i >= WAVE ? 0 : ml & ~((1ull << (st - i)) - 1ull);
            if (!on) ml = 0;
            while (ml) {
                const int pos = (int)__builtin_ctzll(ml);
                ml &= ml - 1ull;
                const int2 et = evs[pos];
                if (m.step(et.x, et.y, cd, a.status)) {
                    m.reset();
                    ++cnt;
                    lastc = i + pos;
                }
            }
        }
    }
    if (on) {
        if (a.count_io) {
            a.count_io[o] += cnt;
            a.last_io[o] = lastc >= 0 ? lastc : prev;
        } else {
            a.out[o] = cnt;
        }
    }
}

template <int N> void deep_n(const DeepArgs &a, hipStream_t s)
{
    const int64_t t0 = a.g0 / WAVE, t1 = (a.g1 + WAVE - 1) / WAVE;
    if (t1 <= t0) return;
    hipLaunchKernelGGL((k_deep<N>), dim3((unsigned)((t1 - t0 + WPB - 1) / WPB)), dim3(WAVE * WPB),
                       0, s, a);
}

template <int N, bool EXACT, int D>
void persist_n(const BatchDev &b, int grid, const int *ctiles, int nct, hipStream_t s, bool fix)
{
    if (fix) {
        if (nct > 0)
            hipLaunchKernelGGL((k_persist_fixup<N, EXACT, D>), dim3((nct + WPB - 1) / WPB),
                               dim3(WAVE * WPB), 0, s, b, ctiles, nct);
    } else {
        const size_t lds = (size_t)b.wpb * 2 * WAVE * sizeof(unsigned long long);
        if (b.sparse)
            hipLaunchKernelGGL((k_persist<N, EXACT, D, true>), dim3(grid), dim3(WAVE * b.wpb),
                               lds, s, b);
        else
            hipLaunchKernelGGL((k_persist<N, EXACT, D, false>), dim3(grid), dim3(WAVE * b.wpb),
                               lds, s, b);
    }
}

template <int N>
void persist_dispatch_n(bool exact, int dcls, const BatchDev &b, int grid, const int *ctiles,
                        int nct, hipStream_t s, bool fix)
{
    if (!exact) return persist_n<N, false, 1>(b, grid, ctiles, nct, s, fix);
    switch (dcls) {
    case 0: return persist_n<N, true, 1>(b, grid, ctiles, nct, s, fix);
    case 1: return persist_n<N, true, 2>(b, grid, ctiles, nct, s, fix);
    case 2: return persist_n<N, true, 4>(b, grid, ctiles, nct, s, fix);
    default: return persist_n<N, true, 8>(b, grid, ctiles, nct, s, fix);
    }
}

template <int N, bool EXACT, int D> void map_n(const MapGroup &g, hipStream_t s, bool fix)
{
    if (fix) {
        hipLaunchKernelGGL((k_fixup<N, EXACT, D>), dim3((unsigned)((g.tiles + WPB - 1) / WPB)),
                           dim3(WAVE * WPB), 0, s, g.ids, g.ticks, g);
    } else if (g.P == 1 && g.sparse) {
        hipLaunchKernelGGL((k_map1<N, EXACT, D, true>),
                           dim3((unsigned)((g.tiles + WPB - 1) / WPB)), dim3(WAVE * WPB), 0, s,
                           g.ids, g.ticks, g);
    } else if (g.P == 1) {
        hipLaunchKernelGGL((k_map1<N, EXACT, D, false>),
                           dim3((unsigned)((g.tiles + WPB - 1) / WPB)), dim3(WAVE * WPB), 0, s,
                           g.ids, g.ticks, g);
    } else {
        const int64_t items = (int64_t)g.tiles * g.P;
        if (g.sparse)
            hipLaunchKernelGGL((k_map<N, EXACT, D, true>),
                               dim3((unsigned)((items + WPB - 1) / WPB)), dim3(WAVE * WPB), 0, s,
                               g.ids, g.ticks, g);
        else
            hipLaunchKernelGGL((k_map<N, EXACT, D, false>),
                               dim3((unsigned)((items + WPB - 1) / WPB)), dim3(WAVE * WPB), 0, s,
                               g.ids, g.ticks, g);
    }
}

template <int N, bool EXACT, int D>
void resume_n(const MapGroup &g, int from, int *count_io, int *last_io, hipStream_t s)
{
    const dim3 grid((unsigned)((g.tiles + WPB - 1) / WPB)), block(WAVE * WPB);
    if (g.sparse)
        hipLaunchKernelGGL((k_resume<N, EXACT, D, true>), grid, block, 0, s, g.ids, g.ticks, g,
                           from, count_io, last_io);
    else
        hipLaunchKernelGGL((k_resume<N, EXACT, D, false>), grid, block, 0, s, g.ids, g.ticks, g,
                           from, count_io, last_io);
}

template <int N>
void resume_dispatch_n(bool exact, int dcls, const MapGroup &g, int from, int *count_io,
                       int *last_io, hipStream_t s)
{
    if (!exact) return resume_n<N, false, 1>(g, from, count_io, last_io, s);
    switch (dcls) {
    case 0: return resume_n<N, true, 1>(g, from, count_io, last_io, s);
    case 1: return resume_n<N, true, 2>(g, from, count_io, last_io, s);
    case 2: return resume_n<N, true, 4>(g, from, count_io, last_io, s);
    default: return resume_n<N, true, 8>(g, from, count_io, last_io, s);
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
