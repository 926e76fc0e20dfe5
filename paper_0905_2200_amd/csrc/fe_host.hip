// fe_host.hip -- host runtime behind include/fe.h: context, workspace,
// candidate grouping, launch planning, two-pass elimination and the
// level-wise mining driver.
#include "fe.h"
#include "fe_hostalgo.h"
#include "fe_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <thread>
#include <vector>

using namespace fe;

namespace {

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
};

// Large host arrays are written in full by the loops that fill them, so they
// are allocated without value-initialisation.  Arrays of 64 MB and more
// (the candidate keys of a big level) go to pinned host memory, so their
// upload is an asynchronous DMA; the mining driver keeps such a buffer for
// reuse, so it is pinned once.
std::mutex g_pin_mu;
std::unordered_map<void *, size_t> g_pinned;  // pinned blocks from NoInit::allocate

template <class T> struct NoInit : std::allocator<T> {
    static constexpr size_t PIN_BYTES = (size_t)64 << 20;
    template <class U> struct rebind {
        typedef NoInit<U> other;
    };
    NoInit() = default;
    template <class U> NoInit(const NoInit<U> &) {}
    T *allocate(size_t n)
    {
        if (n * sizeof(T) >= PIN_BYTES) {
            void *p = nullptr;
            if (hipHostMalloc(&p, n * sizeof(T), hipHostMallocDefault) == hipSuccess && p) {
                std::lock_guard<std::mutex> lk(g_pin_mu);
                g_pinned[p] = n;
                return (T *)p;
            }
            (void)hipGetLastError();
        }
        return std::allocator<T>::allocate(n);
    }
    void deallocate(T *p, size_t n)
    {
        if (n * sizeof(T) >= PIN_BYTES) {
            std::lock_guard<std::mutex> lk(g_pin_mu);
            auto it = g_pinned.find((void *)p);
            if (it != g_pinned.end()) {
                g_pinned.erase(it);
                (void)hipHostFree(p);
                return;
            }
        }
        std::allocator<T>::deallocate(p, n);
    }
    template <class U> void construct(U *p) noexcept { ::new ((void *)p) U; }
    template <class U, class... A> void construct(U *p, A &&...a)
    {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class T, class U> bool operator==(const NoInit<T> &, const NoInit<U> &) { return true; }
template <class T, class U> bool operator!=(const NoInit<T> &, const NoInit<U> &) { return false; }
typedef std::vector<int, NoInit<int>> ivec;
typedef EpisodesT<ivec> Episodes;
typedef HostPackT<ivec> HostPack;

// Fixed device scratch of the no-allocation entry point (fe_count_noalloc):
// each device holds its own copy until the process ends.  Host code never
// uses this name as an address: fe_create looks up this device's copy with
// hipGetSymbolAddress, once per device, and keeps the pointer.
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
std::mutex g_fixed_mu;
std::map<int, char *> g_fixed;  // device -> its copy of scratch

double now_ms()
{
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

constexpr int NPARAM = 16;

struct fe_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int64_t param[NPARAM] = {0, 16384, 1024, 1, 0, 1, 8472, 13112, 2, 0, 0, 9699, 6165, 1000,
                             131072, 1};
    fe_stats stats{};
    // workspace
    Buf keys, hist, wmax, pk, orig, tileW, lam, tbl, flags, sel, nsel, status, small, cmask;
    Buf mtypes, mlen, mlo, mhi, mup, mex, msel, mn, mkey, tscr, tinfo, mfk, mfo, mfsel, pbc;
    Buf deep;  // window rings of the deep-class exact launches
    Buf skey, sup;  // keys and relaxed counts of a level's elimination sample
    // This device's copy of the fixed scratch array (fe_count_noalloc), and
    // while such a call runs, the bump arena its workspace is carved from.
    char *fixed = nullptr;
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    // host arrays of the mining driver, kept for reuse (large ones are pinned)
    ivec keypool, lanepool, uphpool, orderpool;
    int *host = nullptr;  // pinned host staging for small readbacks
    size_t host_cap = 0;
    // kernel timing
    struct Pending {
        std::string name;
        double ee;
        hipEvent_t a, b;
    };
    struct Agg {
        int64_t launches = 0;
        double total_ms = 0, max_ms = 0, ee = 0;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    std::map<std::string, Agg> kstats;
};

namespace {

int fail(fe_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(fe_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(c, x)                                                                   \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess)                                                          \
            return fail((c), FE_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));  \
    } while (0)

int ensure(fe_ctx *c, Buf &b, size_t bytes)
{
    if (bytes == 0) bytes = 4;
    if (c->arena) {
        // no-allocation call: carve from the fixed scratch; never allocate or free
        if (b.p && b.cap >= bytes) return FE_OK;
        const size_t a = (bytes + 255) & ~(size_t)255;
        if (c->arena_used + a > c->arena_cap)
            return fail(c, FE_ENOMEM, "the call needs more than the %zu-byte fixed scratch",
                        c->arena_cap);
        b.p = c->arena + c->arena_used;
        b.cap = a;
        c->arena_used += a;
        return FE_OK;
    }
    if (b.cap >= bytes) return FE_OK;
    if (b.p) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(c, FE_ENOMEM, "device allocation of %zu bytes failed", bytes);
        }
        want = bytes;
    }
    b.cap = want;
    return FE_OK;
}

int ensure_host(fe_ctx *c, size_t ints)
{
    if (c->host_cap >= ints) return FE_OK;
    if (c->arena) return fail(c, FE_EINTERNAL, "pinned staging too small for a no-allocation call");
    if (c->host) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipHostFree(c->host));
        c->host = nullptr;
    }
    if (hipHostMalloc((void **)&c->host, ints * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        c->host = nullptr;
        c->host_cap = 0;
        return fail(c, FE_ENOMEM, "pinned host allocation failed");
    }
    c->host_cap = ints;
    return FE_OK;
}

template <class T> T *P(Buf &b) { return (T *)b.p; }

// ---- kernel timing with HIP events on the context's stream
hipEvent_t pool_event(fe_ctx *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

int resolve_timers(fe_ctx *c)
{
    if (c->pending.empty()) return FE_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
            (void)hipGetLastError();
            ms = 0.f;
        }
        auto &g = c->kstats[p.name];
        g.launches++;
        g.total_ms += ms;
        g.max_ms = std::max(g.max_ms, (double)ms);
        g.ee += p.ee;
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
    return FE_OK;
}

// Scoped timer: records an event before and after the launches in its scope.
struct KTimer {
    fe_ctx *c;
    bool on;
    fe_ctx::Pending p;
    KTimer(fe_ctx *c_, const char *name, double ee)
        : c(c_), on(c_->param[FE_PARAM_TIMING] != 0 && !c_->arena)
    {
        if (!on) return;
        p.name = name;
        p.ee = ee;
        p.a = pool_event(c);
        p.b = pool_event(c);
        if (!p.a || !p.b) { on = false; return; }
        (void)hipEventRecord(p.a, c->stream);
    }
    ~KTimer()
    {
        if (!on) return;
        (void)hipEventRecord(p.b, c->stream);
        c->pending.push_back(p);
        if (c->pending.size() > 4096) (void)resolve_timers(c);
    }
};

int status_code(int bits)
{
    if (bits & ST_BADCAND) return FE_EINVAL;
    if (bits & ST_RANGE) return FE_ERANGE;
    if (bits & ST_UNSORTED) return FE_EUNSORTED;
    if (bits & ST_INTERNAL) return FE_EINTERNAL;
    return FE_OK;
}

const char *status_text(int bits)
{
    if (bits & ST_BADCAND)
        return "invalid candidate (N outside [1,nmax], type outside [0,num_types), "
               "lo<0, lo>=hi, or hi or sum(hi) >= 2^30)";
    if (bits & ST_RANGE) return "event id outside [0,num_types) or tick outside [0,2^30)";
    if (bits & ST_UNSORTED) return "event ticks are not non-decreasing";
    if (bits & ST_INTERNAL) return "internal invariant failed";
    return "ok";
}

struct CandIn {
    const int *types, *len, *lo, *hi;
    int nmax;
};

struct StreamInfo {
    int n;
    int span;       // ticks[n-1] - ticks[0] + 1
    int num_types;  // ids lie in [0, num_types) (validated)
};

// Segment count P for a group of `tiles` tiles of N-node candidates: the
// hybrid rule of Algorithm 2 (Eq. 2).  The whole-stream Map (the paper's
// PTPE, P = 1) once the tiles reach the crossover C(N) = a/N + b tiles,
// else MapConcatenate with P >= 2 segments, enough for the target number of
// waves, each segment long against the look-back (about n*W/span events).
// a and b were fitted, per counter, to measured crossovers on a 256-CU
// MI355X (paper_0905_2200_amd/crossover.py), as the paper fits its Table 1
// with a/N + b.
int choose_P(const fe_ctx *c, int tiles, const StreamInfo &si, int Wmax, int N, bool exact)
{
    const int n = si.n;
    if (n <= 1) return 1;
    if (c->param[FE_PARAM_SEGMENTS] > 0)
        return (int)std::min<int64_t>(c->param[FE_PARAM_SEGMENTS], n);
    const int pa = exact ? FE_PARAM_CROSSOVER_A : FE_PARAM_CROSSOVER_A_RELAXED;
    const int pb = exact ? FE_PARAM_CROSSOVER_B : FE_PARAM_CROSSOVER_B_RELAXED;
    const double cross = (double)c->param[pa] / std::max(N, 1) + (double)c->param[pb];
    if ((double)tiles >= cross) return 1;
    const int64_t target = c->param[FE_PARAM_TARGET_WAVES];
    int64_t P = std::max<int64_t>(2, (target + tiles - 1) / std::max(tiles, 1));
    const double lb = (double)n * (double)Wmax / std::max(si.span, 1);
    const int64_t minseg = std::max<int64_t>(c->param[FE_PARAM_MIN_SEG_EVENTS],
                                             (int64_t)(8.0 * lb) + 64);
    P = std::min<int64_t>(P, std::max<int64_t>(1, n / minseg));
    P = std::min<int64_t>(P, 4096);
    return (int)std::max<int64_t>(P, 1);
}

// Launch plan of a deep-class group over a stream of n events: each lane's
// N-1 lists hold cap = min(dcap, n) windows (live windows of a list number at
// most its hop's window bound, and at most the events of the range
// [t - hi, t]); lanes are processed in chunks whose rings fit the scratch
// budget (at least one lane per chunk).
struct DeepPlan {
    int cap = 1;
    int64_t chunk = 0;   // lanes per launch
    int64_t bytes = 0;   // ring bytes of one launch
};

DeepPlan deep_plan(int N, int64_t lanes, int dcap, int n, int64_t budget = DEEP_SCRATCH)
{
    DeepPlan p;
    p.cap = std::max(1, std::min(dcap, std::max(n, 1)));
    const int64_t per = (int64_t)std::max(N - 1, 1) * p.cap * (int64_t)sizeof(int2);
    p.chunk = std::max<int64_t>(1, std::min<int64_t>(lanes, budget / per));
    if (p.chunk >= WAVE) p.chunk = p.chunk / WAVE * WAVE;
    p.bytes = p.chunk * per;
    return p;
}

// Enqueue the chunks of a deep-class group (a: everything but the lane range
// and the ring capacity); `lanes` = the group's tiles * 64.
void deep_launch(int N, DeepArgs a, const DeepPlan &p, int64_t lanes, hipStream_t s)
{
    a.cap = p.cap;
    for (int64_t g0 = 0; g0 < lanes; g0 += p.chunk) {
        a.g0 = g0;
        a.g1 = std::min(lanes, g0 + p.chunk);
        launch_deep(N, a, s);
    }
}

// Incremental count (fe_count_resume): events before `from` were counted by
// earlier calls; per candidate, count_io / last_io carry the count and the
// index of the last completion so far.
struct Resume {
    int from;
    int *count_io, *last_io;
};

// Map (+ plan, Concatenate, fix-up when segmented) for every packed group;
// with rs, the incremental whole-stream Map instead.
int launch_groups(fe_ctx *c, const int *ids, const int *ticks, const StreamInfo &si,
                  const std::vector<GroupDesc> &groups, bool exact, int *out,
                  const Resume *rs = nullptr, const char *tag = "map")
{
    hipStream_t s = c->stream;
    int rc;
    const unsigned long long *cmask = nullptr;
    if (si.n > 0) {
        if ((rc = ensure(c, c->cmask, (size_t)((si.n + 7) / 8) * sizeof(unsigned long long))))
            return rc;
        launch_chunkmask(ids, si.n, (unsigned long long *)c->cmask.p, s);
        cmask = (const unsigned long long *)c->cmask.p;
    }
    for (const GroupDesc &gd : groups) {
        const int k = gd.key;
        const int N = k / NDCLS + 1, dcls = k % NDCLS;
        const int tiles = gd.tiles;
        if (exact && dcls == DEEP_CLS) {
            // lists beyond 8 windows: rings in device memory, whole stream
            const int64_t lanes = (int64_t)tiles * WAVE;
            const int64_t budget =
                c->arena ? (int64_t)(c->arena_cap - c->arena_used) / 256 * 256 : DEEP_SCRATCH;
            const DeepPlan dp = deep_plan(N, lanes, gd.dcap, si.n, std::max<int64_t>(budget, 1));
            if ((rc = ensure(c, c->deep, (size_t)dp.bytes))) return rc;
            DeepArgs a{};
            a.ids = ids;
            a.ticks = ticks;
            a.n = si.n;
            a.pk = P<int>(c->pk) + gd.rec_base;
            a.orig = P<int>(c->orig) + (int64_t)gd.tile_base * WAVE;
            a.ring = P<int2>(c->deep);
            a.out = out;
            a.status = P<int>(c->status);
            if (rs) {
                a.from = rs->from;
                a.count_io = rs->count_io;
                a.last_io = rs->last_io;
            }
            c->stats.map_launches++;
            char dname[40];
            snprintf(dname, sizeof dname, "%s_exact_n%d_deep", rs ? "resume" : "map", N);
            KTimer kt(c, dname, (double)gd.ncand * (double)(si.n - (rs ? rs->from : 0)));
            deep_launch(N, a, dp, lanes, s);
            HIPCHK(c, hipGetLastError());
            continue;
        }
        MapGroup g;
        g.ids = ids;
        g.ticks = ticks;
        g.n = si.n;
        g.pk = P<int>(c->pk) + gd.rec_base;
        g.orig = P<int>(c->orig) + (int64_t)gd.tile_base * WAVE;
        g.out = out;
        g.status = P<int>(c->status);
        g.cmask = cmask;
        g.tiles = tiles;
        g.lam = nullptr;
        g.tbl = nullptr;
        g.flags = nullptr;
        g.P = rs ? 1 : choose_P(c, tiles, si, gd.wmax, N, exact);
        if (c->arena) {
            // no-allocation call: as many segments as the fixed scratch's
            // remainder holds the tables of (P = 1 needs none)
            const size_t avail = c->arena_cap - c->arena_used;
            auto need = [&](int64_t P) {
                const auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
                return al((size_t)tiles * (P + 1) * sizeof(int)) +
                       al((size_t)P * tiles * WAVE * KMAX * sizeof(int2)) +
                       al((size_t)tiles * WAVE * sizeof(int));
            };
            while (g.P > 1 && need(g.P) > avail) g.P /= 2;
        }
        g.sparse = c->param[FE_PARAM_TYPE_DISPATCH] != 0;
        g.hashx = si.num_types <= 64;
        g.shlists = c->param[FE_PARAM_SHARED_LISTS] != 0;
        c->stats.map_launches++;
        if (rs) {
            char rname[40];
            snprintf(rname, sizeof rname, "resume_%s_n%d_d%d", exact ? "exact" : "relaxed", N,
                     exact ? dcls_depth(dcls) : 1);
            KTimer kt(c, rname, (double)gd.ncand * (double)(si.n - rs->from));
            launch_resume(N, exact, dcls, g, rs->from, rs->count_io, rs->last_io, s);
            HIPCHK(c, hipGetLastError());
            continue;
        }
        char kname[40];
        snprintf(kname, sizeof kname, "%s_%s_n%d_d%d", tag, exact ? "exact" : "relaxed", N,
                 exact ? dcls_depth(dcls) : 1);
        const double ee = (double)gd.ncand * (double)si.n;
        c->stats.segments_max = std::max<int64_t>(c->stats.segments_max, g.P);
        if (g.P > 1) {
            const int64_t lam_n = (int64_t)tiles * (g.P + 1);
            const int64_t tbl_n = (int64_t)g.P * tiles * WAVE * KMAX;
            if ((rc = ensure(c, c->lam, (size_t)lam_n * sizeof(int)))) return rc;
            if ((rc = ensure(c, c->tbl, (size_t)tbl_n * sizeof(int2)))) return rc;
            if ((rc = ensure(c, c->flags, (size_t)tiles * WAVE * sizeof(int)))) return rc;
            g.lam = P<int>(c->lam);
            g.tbl = P<int2>(c->tbl);
            g.flags = P<int>(c->flags);
            {
                KTimer kt(c, "plan", 0);
                launch_fill(g.flags, 0, (int64_t)tiles * WAVE, s);
                launch_plan(ticks, si.n, P<int>(c->tileW) + gd.tile_base, tiles, g.P,
                            P<int>(c->lam), s);
            }
            {
                KTimer kt(c, kname, ee);
                launch_map(N, exact, dcls, g, s);
            }
            {
                const bool tree = c->param[FE_PARAM_CONCAT_TREE] && g.P >= 16;
                KTimer kt(c, tree ? "concat_tree" : "concat_seq", 0);
                launch_concat(g, tree, s);
            }
            {
                KTimer kt(c, "fixup", 0);
                launch_fixup(N, exact, dcls, g, s);
            }
        } else {
            KTimer kt(c, kname, ee);
            launch_map(N, exact, dcls, g, s);
        }
        HIPCHK(c, hipGetLastError());
    }
    return FE_OK;
}

// One counting pass (relaxed or exact) over candidates cin (optionally the
// subset sel[0..*nsel) of them), writing out[m] for every counted m.
int run_pass(fe_ctx *c, const int *ids, const int *ticks, const StreamInfo &si, int num_types,
             const CandIn &cin, const int *sel, const int *nsel, int M, bool exact, int *out,
             const Resume *rs = nullptr)
{
    hipStream_t s = c->stream;
    int rc;
    if ((rc = ensure(c, c->keys, (size_t)M * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->hist, 3 * NKEYS * sizeof(int)))) return rc;
    // per-block key counts and their scan (stable placement in key groups)
    const int64_t nbc = (int64_t)NKEYS * ((M + 255) / 256);
    if ((rc = ensure(c, c->pbc, (size_t)(2 * nbc + scan_scratch_ints(nbc)) * sizeof(int))))
        return rc;
    int *bcnt = P<int>(c->pbc), *boff = bcnt + nbc;
    int *hist = P<int>(c->hist);
    launch_fill(hist, 0, 3 * NKEYS, s);
    {
        KTimer kt(c, "prep_count", 0);
        launch_prep_count(cin.types, cin.len, cin.lo, cin.hi, cin.nmax, sel, nsel, M, num_types,
                          exact ? 1 : 0, P<int>(c->keys), hist, P<int>(c->status), bcnt, s);
        launch_scan_excl(bcnt, nbc, boff, boff + nbc, s);
    }
    if ((rc = ensure_host(c, 3 * NKEYS + 1))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->host, hist, 3 * NKEYS * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->host + 3 * NKEYS, P<int>(c->status), sizeof(int),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    const int bits = c->host[3 * NKEYS];
    if (bits) {
        launch_fill(P<int>(c->status), 0, 1, s);
        return fail(c, status_code(bits), "%s", status_text(bits));
    }
    int cnt[NKEYS], wmax[NKEYS], bmax[NKEYS];
    std::memcpy(cnt, c->host, sizeof cnt);
    std::memcpy(wmax, c->host + NKEYS, sizeof wmax);
    std::memcpy(bmax, c->host + 2 * NKEYS, sizeof bmax);

    Layout lay;
    int tiles_total = 0;
    int64_t rec_total = 0;
    for (int k = 0; k < NKEYS; ++k) {
        const int N = k / NDCLS + 1;
        const int t = (cnt[k] + WAVE - 1) / WAVE;
        lay.tile_base[k] = tiles_total;
        lay.rec_base[k] = (int)rec_total;
        tiles_total += t;
        rec_total += (int64_t)t * rec_ints(N);
    }
    if (rec_total >= (int64_t)1 << 31)
        return fail(c, FE_EINVAL, "candidate table too large (%lld ints)", (long long)rec_total);
    if (tiles_total == 0) return FE_OK;
    if ((rc = ensure(c, c->pk, (size_t)rec_total * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->orig, (size_t)tiles_total * WAVE * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->tileW, (size_t)tiles_total * sizeof(int)))) return rc;
    {
        KTimer kt(c, "prep_scatter", 0);
        launch_fill(P<int>(c->pk), -1, rec_total, s);
        launch_fill(P<int>(c->orig), -1, (int64_t)tiles_total * WAVE, s);
        launch_fill(P<int>(c->tileW), 0, tiles_total, s);
        launch_prep_scatter(cin.types, cin.len, cin.lo, cin.hi, cin.nmax, sel, nsel, M,
                            P<int>(c->keys), lay, boff, P<int>(c->pk),
                            P<int>(c->orig), P<int>(c->tileW), s);
    }

    std::vector<GroupDesc> groups;
    for (int k = 0; k < NKEYS; ++k)
        if (cnt[k])
            groups.push_back(GroupDesc{k, (cnt[k] + WAVE - 1) / WAVE, lay.tile_base[k],
                                       (int64_t)lay.rec_base[k], wmax[k], (int64_t)cnt[k],
                                       bmax[k]});
    return launch_groups(c, ids, ticks, si, groups, exact, out, rs);
}

int check_common(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                 int32_t num_types)
{
    if (!c) return FE_EINVAL;
    if (n < 0 || n >= ((int64_t)1 << 31) - 64) return fail(c, FE_EINVAL, "n out of range");
    if (n > 0 && (!ids || !ticks)) return fail(c, FE_EINVAL, "null stream pointer");
    if (num_types <= 0) return fail(c, FE_EINVAL, "num_types must be positive");
    return FE_OK;
}

int check_cands(fe_ctx *c, const int32_t *types, const int32_t *len, const int32_t *lo,
                const int32_t *hi, int32_t M, int32_t nmax)
{
    if (M < 0) return fail(c, FE_EINVAL, "M < 0");
    if (nmax < 1 || nmax > NMAX) return fail(c, FE_EINVAL, "nmax outside [1,8]");
    if (M > 0 && (!types || !len || (nmax > 1 && (!lo || !hi))))
        return fail(c, FE_EINVAL, "null candidate pointer");
    if ((int64_t)M * nmax >= ((int64_t)1 << 31)) return fail(c, FE_EINVAL, "M too large");
    return FE_OK;
}

// Validate the stream and learn its tick span (synchronises).
int stream_info(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int n, int num_types,
                StreamInfo &si)
{
    int rc;
    si.n = n;
    si.span = 1;
    si.num_types = num_types;
    if (n == 0) return FE_OK;
    launch_validate(ids, ticks, n, num_types, P<int>(c->status), c->stream);
    if ((rc = ensure_host(c, 4))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->host, ticks, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->host + 1, ticks + (n - 1), sizeof(int), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->host + 2, P<int>(c->status), sizeof(int),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int bits = c->host[2];
    if (bits) {
        launch_fill(P<int>(c->status), 0, 1, c->stream);
        return fail(c, status_code(bits), "%s", status_text(bits));
    }
    si.span = std::max(1, c->host[1] - c->host[0] + 1);
    return FE_OK;
}

int count_impl(fe_ctx *c, const int32_t *ids, const int32_t *ticks, const StreamInfo &si,
               int32_t num_types, const CandIn &cin, int32_t M, int mode, int32_t *out)
{
    if (M == 0) return FE_OK;
    if (si.n == 0) {
        launch_fill(out, 0, M, c->stream);
        return FE_OK;
    }
    return run_pass(c, ids, ticks, si, num_types, cin, nullptr, nullptr, M, mode == FE_EXACT,
                    out);
}

int two_pass_impl(fe_ctx *c, const int32_t *ids, const int32_t *ticks, const StreamInfo &si,
                  int32_t num_types, const CandIn &cin, int32_t M, int32_t theta,
                  int32_t *upper, int32_t *exact, int32_t *nsurv_out)
{
    int rc;
    hipStream_t s = c->stream;
    if ((rc = ensure(c, c->nsel, sizeof(int)))) return rc;
    launch_fill(P<int>(c->nsel), 0, 1, s);
    if (M == 0) {
        if (nsurv_out)
            HIPCHK(c, hipMemcpyAsync(nsurv_out, P<int>(c->nsel), sizeof(int),
                                     hipMemcpyDeviceToDevice, s));
        return FE_OK;
    }
    if ((rc = count_impl(c, ids, ticks, si, num_types, cin, M, FE_RELAXED, upper))) return rc;
    if ((rc = ensure(c, c->sel, (size_t)M * sizeof(int)))) return rc;
    // empty stream: every count is 0, so kept candidates keep exact = 0
    if (si.n == 0) launch_fill(exact, 0, M, s);
    {
        KTimer kt(c, "compact", 0);
        launch_compact(upper, M, theta, exact, P<int>(c->sel), P<int>(c->nsel), s);
    }
    if (si.n > 0) {
        int ns = 0;
        HIPCHK(c, hipMemcpyAsync(c->host, P<int>(c->nsel), sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        ns = c->host[0];
        if ((int64_t)ns * 2 > (int64_t)M) {
            // most candidates survive: count them all in their input order
            // (which keeps tiles of join siblings together) and keep the
            // survivors' counts
            if ((rc = ensure(c, c->small, (size_t)M * sizeof(int)))) return rc;
            if ((rc = run_pass(c, ids, ticks, si, num_types, cin, nullptr, nullptr, M, true,
                               P<int>(c->small))))
                return rc;
            launch_select(upper, P<int>(c->small), M, theta, exact, s);
        } else if (ns > 0) {
            if ((rc = run_pass(c, ids, ticks, si, num_types, cin, P<int>(c->sel), P<int>(c->nsel),
                               M, true, exact)))
                return rc;
        }
    }
    if (nsurv_out)
        HIPCHK(c, hipMemcpyAsync(nsurv_out, P<int>(c->nsel), sizeof(int), hipMemcpyDeviceToDevice,
                                 s));
    return FE_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" int fe_create(int device, void *hip_stream, fe_ctx **out)
{
    if (!out) return FE_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return FE_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return FE_EDEVICE;
    fe_ctx *c = new (std::nothrow) fe_ctx();
    if (!c) return FE_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;  // NULL: the device's null stream
    c->own_stream = false;
    if (ensure(c, c->status, sizeof(int)) || ensure_host(c, 256)) {
        fe_destroy(c);
        return FE_ENOMEM;
    }
    launch_fill(P<int>(c->status), 0, 1, c->stream);
    {
        // this device's copy of the fixed scratch (with the device current)
        std::lock_guard<std::mutex> lk(g_fixed_mu);
        auto it = g_fixed.find(device);
        if (it == g_fixed.end()) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e == hipSuccess && p) it = g_fixed.emplace(device, (char *)p).first;
            else (void)hipGetLastError();
        }
        if (it != g_fixed.end()) c->fixed = it->second;
    }
    *out = c;
    return FE_OK;
}

extern "C" int fe_destroy(fe_ctx *c)
{
    if (!c) return FE_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    Buf *bufs[] = {&c->keys, &c->hist, &c->wmax, &c->pk,    &c->orig,  &c->tileW,
                   &c->lam,  &c->tbl,  &c->flags, &c->sel, &c->nsel,  &c->status, &c->small, &c->cmask,
                   &c->mtypes, &c->mlen, &c->mlo, &c->mhi, &c->mup, &c->mex, &c->msel, &c->mn,
                   &c->mkey, &c->tscr, &c->tinfo, &c->mfk, &c->mfo, &c->mfsel, &c->pbc,
                   &c->deep, &c->skey, &c->sup};
    for (Buf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    if (c->host) (void)hipHostFree(c->host);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return FE_OK;
}

extern "C" const char *fe_last_error(const fe_ctx *c)
{
    return c ? c->err.c_str() : "null context";
}

extern "C" int fe_sync(fe_ctx *c)
{
    if (!c) return FE_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(c->host, P<int>(c->status), sizeof(int), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    const int bits = c->host[0];
    if (bits) {
        launch_fill(P<int>(c->status), 0, 1, c->stream);
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return fail(c, status_code(bits), "%s", status_text(bits));
    }
    return FE_OK;
}

extern "C" int fe_set_param(fe_ctx *c, int param, int64_t value)
{
    if (!c) return FE_EINVAL;
    const bool signed_ok = param == FE_PARAM_CROSSOVER_A || param == FE_PARAM_CROSSOVER_A_RELAXED;
    if (param < 0 || param >= NPARAM || (value < 0 && !signed_ok))
        return fail(c, FE_EINVAL, "bad parameter");
    if (param == FE_PARAM_ELIMINATION && value > 2) return fail(c, FE_EINVAL, "bad parameter");
    if (param == FE_PARAM_TARGET_WAVES && value == 0) return fail(c, FE_EINVAL, "bad parameter");
    c->param[param] = value;
    return FE_OK;
}

extern "C" int fe_get_param(const fe_ctx *c, int param, int64_t *value)
{
    if (!c || !value || param < 0 || param >= NPARAM) return FE_EINVAL;
    *value = c->param[param];
    return FE_OK;
}

extern "C" int fe_get_stats(const fe_ctx *c, fe_stats *out)
{
    if (!c || !out) return FE_EINVAL;
    *out = c->stats;
    return FE_OK;
}

extern "C" int fe_get_kernel_stats(fe_ctx *c, fe_kernel_stat *out, int32_t cap, int32_t *n_out)
{
    if (!c || !n_out || cap < 0 || (cap > 0 && !out)) return FE_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    if ((rc = resolve_timers(c))) return rc;
    int i = 0;
    for (auto &kv : c->kstats) {
        if (i < cap) {
            fe_kernel_stat &o = out[i];
            std::memset(&o, 0, sizeof o);
            std::snprintf(o.name, sizeof o.name, "%s", kv.first.c_str());
            o.launches = kv.second.launches;
            o.total_ms = kv.second.total_ms;
            o.max_ms = kv.second.max_ms;
            o.ee = kv.second.ee;
        }
        ++i;
    }
    *n_out = i;
    return FE_OK;
}

extern "C" int fe_reset_kernel_stats(fe_ctx *c)
{
    if (!c) return FE_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    if ((rc = resolve_timers(c))) return rc;
    c->kstats.clear();
    return FE_OK;
}

extern "C" int fe_validate(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                           int32_t num_types)
{
    int rc;
    if ((rc = check_common(c, ids, ticks, n, num_types))) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    StreamInfo si;
    return stream_info(c, ids, ticks, (int)n, num_types, si);
}

extern "C" int fe_count(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                        int32_t num_types, const int32_t *types, const int32_t *len,
                        const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax, int mode,
                        int32_t *counts_out)
{
    int rc;
    const double t0 = now_ms();
    if ((rc = check_common(c, ids, ticks, n, num_types))) return rc;
    if ((rc = check_cands(c, types, len, lo, hi, M, nmax))) return rc;
    if (mode != FE_EXACT && mode != FE_RELAXED) return fail(c, FE_EINVAL, "bad mode");
    if (M > 0 && !counts_out) return fail(c, FE_EINVAL, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    c->stats = fe_stats{};
    StreamInfo si;
    if ((rc = stream_info(c, ids, ticks, (int)n, num_types, si))) return rc;
    CandIn cin{types, len, lo, hi, nmax};
    rc = count_impl(c, ids, ticks, si, num_types, cin, M, mode, counts_out);
    c->stats.last_call_ms = now_ms() - t0;
    return rc;
}

extern "C" int fe_count_noalloc(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                                int32_t num_types, const int32_t *types, const int32_t *len,
                                const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax,
                                int mode, int32_t *counts_out)
{
    int rc;
    const double t0 = now_ms();
    if ((rc = check_common(c, ids, ticks, n, num_types))) return rc;
    if ((rc = check_cands(c, types, len, lo, hi, M, nmax))) return rc;
    if (mode != FE_EXACT && mode != FE_RELAXED) return fail(c, FE_EINVAL, "bad mode");
    if (M > 0 && !counts_out) return fail(c, FE_EINVAL, "null output");
    if (!c->fixed) return fail(c, FE_EDEVICE, "no fixed scratch on device %d", c->device);
    // the workspace of a whole-stream count (P = 1, no deep rings) must fit
    const auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t tiles_max = ((int64_t)M + WAVE - 1) / WAVE + NKEYS;
    const int64_t nbc = (int64_t)NKEYS * ((M + 255) / 256);
    const size_t need = al((size_t)M * 4) + al(3 * NKEYS * 4) +
                        al((size_t)(2 * nbc + scan_scratch_ints(nbc)) * 4) +
                        al((size_t)tiles_max * rec_ints(nmax) * 4) +
                        al((size_t)tiles_max * WAVE * 4) + al((size_t)tiles_max * 4) +
                        al((size_t)((n + 7) / 8) * 8);
    if (need > NOALLOC_BYTES)
        return fail(c, FE_ENOMEM,
                    "%d candidates over %lld events need up to %zu bytes of workspace; the "
                    "fixed scratch holds %zu (use fe_count)",
                    M, (long long)n, need, NOALLOC_BYTES);
    HIPCHK(c, hipSetDevice(c->device));
    c->stats = fe_stats{};
    // every workspace buffer of the call comes from the fixed scratch; the
    // context's own buffers are set aside and restored afterwards
    Buf *ws[] = {&c->keys, &c->hist, &c->pbc, &c->pk,  &c->orig, &c->tileW,
                 &c->cmask, &c->lam, &c->tbl, &c->flags, &c->deep};
    constexpr int NWS = (int)(sizeof ws / sizeof ws[0]);
    Buf saved[NWS];
    for (int i = 0; i < NWS; ++i) {
        saved[i] = *ws[i];
        *ws[i] = Buf{};
    }
    c->arena = c->fixed;
    c->arena_cap = NOALLOC_BYTES;
    c->arena_used = 0;
    StreamInfo si;
    rc = stream_info(c, ids, ticks, (int)n, num_types, si);
    if (!rc) {
        CandIn cin{types, len, lo, hi, nmax};
        rc = count_impl(c, ids, ticks, si, num_types, cin, M, mode, counts_out);
    }
    c->arena = nullptr;
    for (int i = 0; i < NWS; ++i) *ws[i] = saved[i];
    c->stats.last_call_ms = now_ms() - t0;
    return rc;
}

extern "C" int fe_count_two_pass(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                                 int32_t num_types, const int32_t *types, const int32_t *len,
                                 const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax,
                                 int32_t theta, int32_t *upper_out, int32_t *exact_out,
                                 int32_t *n_survivors_out)
{
    int rc;
    const double t0 = now_ms();
    if ((rc = check_common(c, ids, ticks, n, num_types))) return rc;
    if ((rc = check_cands(c, types, len, lo, hi, M, nmax))) return rc;
    if (M > 0 && (!upper_out || !exact_out)) return fail(c, FE_EINVAL, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    c->stats = fe_stats{};
    StreamInfo si;
    if ((rc = stream_info(c, ids, ticks, (int)n, num_types, si))) return rc;
    CandIn cin{types, len, lo, hi, nmax};
    rc = two_pass_impl(c, ids, ticks, si, num_types, cin, M, theta, upper_out, exact_out,
                       n_survivors_out);
    c->stats.last_call_ms = now_ms() - t0;
    return rc;
}

extern "C" int fe_count_resume(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                               int32_t num_types, const int32_t *types, const int32_t *len,
                               const int32_t *lo, const int32_t *hi, int32_t M, int32_t nmax,
                               int mode, int64_t from, int32_t *count_io, int32_t *last_io)
{
    int rc;
    const double t0 = now_ms();
    if ((rc = check_common(c, ids, ticks, n, num_types))) return rc;
    if ((rc = check_cands(c, types, len, lo, hi, M, nmax))) return rc;
    if (mode != FE_EXACT && mode != FE_RELAXED) return fail(c, FE_EINVAL, "bad mode");
    if (from < 0 || from > n) return fail(c, FE_EINVAL, "from outside [0, n]");
    if (M > 0 && (!count_io || !last_io)) return fail(c, FE_EINVAL, "null carry arrays");
    HIPCHK(c, hipSetDevice(c->device));
    c->stats = fe_stats{};
    StreamInfo si;
    if ((rc = stream_info(c, ids, ticks, (int)n, num_types, si))) return rc;
    if (M > 0 && from < n) {
        CandIn cin{types, len, lo, hi, nmax};
        const Resume rs{(int)from, count_io, last_io};
        rc = run_pass(c, ids, ticks, si, num_types, cin, nullptr, nullptr, M, mode == FE_EXACT,
                      nullptr, &rs);
    }
    c->stats.last_call_ms = now_ms() - t0;
    return rc;
}

// ====================================================================== mining

namespace {


// Host phase timer: with FE_PARAM_TIMING on, adds the wall time of its scope
// to the per-kind table under `name` (a host phase, no device work).
struct HTimer {
    fe_ctx *c;
    const char *name;
    double t0;
    HTimer(fe_ctx *c_, const char *name_) : c(c_), name(name_), t0(now_ms()) {}
    ~HTimer()
    {
        if (!c->param[FE_PARAM_TIMING]) return;
        auto &g = c->kstats[name];
        const double ms = now_ms() - t0;
        g.launches++;
        g.total_ms += ms;
        g.max_ms = std::max(g.max_ms, ms);
    }
};

struct LevelOut {
    int level;
    int64_t ncand, nsurv, nfreq;
    std::vector<int> types, lo, hi, upper, exact;
    double gen_ms, count_ms;
    int passes = 2;
    int64_t sample_n = 0, sample_kept = 0;
    // every candidate (FE_PARAM_KEEP_CANDIDATES)
    std::vector<int> all_types, all_lo, all_hi, all_upper, all_exact;
};

// keys (E1, lo1, hi1, E2, ...) of m-node episodes to types / lo / hi rows
void split_keys(const int *key, size_t cnt, int m, std::vector<int> &ty, std::vector<int> &lo,
                std::vector<int> &hi)
{
    ty.resize(cnt * m);
    lo.resize(cnt * (m - 1));
    hi.resize(cnt * (m - 1));
    const int w = 3 * m - 2;
    for (size_t i = 0; i < cnt; ++i) {
        const int *k = key + i * w;
        for (int j = 0; j < m; ++j) ty[i * m + j] = k[3 * j];
        for (int j = 0; j < m - 1; ++j) {
            lo[i * (m - 1) + j] = k[3 * j + 1];
            hi[i * (m - 1) + j] = k[3 * j + 2];
        }
    }
}

// Lanes-only pack: upload the lane assignment and build the tile records
// and look-back widths on the device from the level's keys (key_d).
int upload_lanes(fe_ctx *c, const HostPack &hp, const int *key_d, int m)
{
    int rc;
    hipStream_t s = c->stream;
    const size_t tiles = (size_t)hp.tiles;
    if ((rc = ensure(c, c->pk, std::max<size_t>(tiles * rec_ints(m), 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->orig, std::max<size_t>(hp.orig.size(), 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->tileW, std::max<size_t>(tiles, 1) * sizeof(int)))) return rc;
    HIPCHK(c, hipStreamSynchronize(s));
    if (!hp.orig.empty())
        HIPCHK(c, hipMemcpyAsync(P<int>(c->orig), hp.orig.data(), hp.orig.size() * sizeof(int),
                                 hipMemcpyHostToDevice, s));
    launch_build_rec(key_d, m, P<int>(c->orig), (int)tiles, P<int>(c->pk), P<int>(c->tileW), s);
    HIPCHK(c, hipGetLastError());
    return FE_OK;
}

int upload_pack(fe_ctx *c, const HostPack &hp)
{
    int rc;
    hipStream_t s = c->stream;
    if ((rc = ensure(c, c->pk, std::max<size_t>(hp.rec.size(), 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->orig, std::max<size_t>(hp.orig.size(), 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->tileW, std::max<size_t>(hp.tileW.size(), 1) * sizeof(int)))) return rc;
    HIPCHK(c, hipStreamSynchronize(s));
    if (!hp.rec.empty())
        HIPCHK(c, hipMemcpyAsync(P<int>(c->pk), hp.rec.data(), hp.rec.size() * sizeof(int),
                                 hipMemcpyHostToDevice, s));
    if (!hp.orig.empty())
        HIPCHK(c, hipMemcpyAsync(P<int>(c->orig), hp.orig.data(), hp.orig.size() * sizeof(int),
                                 hipMemcpyHostToDevice, s));
    if (!hp.tileW.empty())
        HIPCHK(c, hipMemcpyAsync(P<int>(c->tileW), hp.tileW.data(),
                                 hp.tileW.size() * sizeof(int), hipMemcpyHostToDevice, s));
    return FE_OK;
}

// Device tiling of a level (fe_tiling.hip): lanes, records and look-back
// widths of the candidates kept (all, or upper >= theta when up is set),
// grouped by list-depth class when exact.  kept: their number.
int dev_pack(fe_ctx *c, const int *key_d, int m, int64_t M, const int *up, int theta,
             bool exact, int wbound, int bbound, std::vector<GroupDesc> &groups, int64_t &kept)
{
    int rc;
    hipStream_t s = c->stream;
    groups.clear();
    kept = 0;
    constexpr int NINFO = 5 * NDCLS + 1;
    if ((rc = ensure(c, c->tscr, (size_t)tile_scratch_ints(M) * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->tinfo, NINFO * sizeof(int)))) return rc;
    if ((rc = ensure_host(c, NINFO))) return rc;
    {
        KTimer kt(c, "tile_plan", 0);
        launch_tile_plan(key_d, m, M, up, theta, exact, P<int>(c->tscr), P<int>(c->tinfo), s);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->host, P<int>(c->tinfo), NINFO * sizeof(int),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    int info[NINFO];
    std::memcpy(info, c->host, sizeof info);
    const int64_t tiles = info[5 * NDCLS];
    for (int k = 0; k < NDCLS; ++k) kept += info[4 * NDCLS + k];
    if (tiles == 0) return FE_OK;
    const int ri = rec_ints(m);
    if ((rc = ensure(c, c->pk, (size_t)tiles * ri * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->orig, (size_t)tiles * WAVE * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->tileW, (size_t)tiles * sizeof(int)))) return rc;
    launch_fill(P<int>(c->orig), -1, tiles * WAVE, s);
    {
        KTimer kt(c, "tile_lanes", 0);
        launch_tile_lanes(M, P<int>(c->tscr), P<int>(c->tinfo), P<int>(c->orig), s);
    }
    launch_build_rec(key_d, m, P<int>(c->orig), (int)tiles, P<int>(c->pk), P<int>(c->tileW), s);
    HIPCHK(c, hipGetLastError());
    for (int k = 0; k < NDCLS; ++k)
        if (info[k] > 0)
            groups.push_back(GroupDesc{(m - 1) * NDCLS + k, info[k], info[NDCLS + k],
                                       (int64_t)info[NDCLS + k] * ri, wbound,
                                       (int64_t)info[4 * NDCLS + k], bbound});
    return FE_OK;
}

// The elimination decision of a level (FE_PARAM_ELIMINATION = 2): the
// relaxed pass over a sample of the level's candidates (every 64th block of
// 64 consecutive ones, so join siblings stay together); ns sampled, nk of
// them with upper >= theta.
int sample_survival(fe_ctx *c, const int *ids, const int *ticks, const StreamInfo &si, int level,
                    int64_t M, int wbound, int bbound, int theta, int64_t &ns, int64_t &nk)
{
    int rc;
    hipStream_t s = c->stream;
    const int wk = 3 * level - 2;
    ns = sample_count(M);
    nk = 0;
    if (ns <= 0) return FE_OK;
    if ((rc = ensure(c, c->skey, (size_t)ns * wk * sizeof(int)))) return rc;
    if ((rc = ensure(c, c->sup, (size_t)ns * sizeof(int)))) return rc;
    launch_sample_keys(P<int>(c->mkey), wk, M, P<int>(c->skey), s);
    std::vector<GroupDesc> groups;
    int64_t kept = 0;
    if ((rc = dev_pack(c, P<int>(c->skey), level, ns, nullptr, 0, false, wbound, bbound, groups,
                       kept)))
        return rc;
    if ((rc = launch_groups(c, ids, ticks, si, groups, false, P<int>(c->sup), nullptr, "sample")))
        return rc;
    launch_fill(P<int>(c->mn), 0, 1, s);
    launch_compact(P<int>(c->sup), (int)ns, theta, nullptr, P<int>(c->msel), P<int>(c->mn), s);
    HIPCHK(c, hipMemcpyAsync(c->host, P<int>(c->mn), sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    nk = c->host[0];
    return FE_OK;
}

}  // namespace

extern "C" int fe_mine(fe_ctx *c, const int32_t *ids, const int32_t *ticks, int64_t n,
                       int32_t num_types, const int32_t *iv_lo, const int32_t *iv_hi, int32_t n_iv,
                       int32_t theta, int32_t max_level, fe_result **out)
{
    int rc;
    const double t_call = now_ms();
    if (!out) return fail(c, FE_EINVAL, "null result pointer");
    *out = nullptr;
    if ((rc = check_common(c, ids, ticks, n, num_types))) return rc;
    if (max_level < 1 || max_level > NMAX) return fail(c, FE_EINVAL, "max_level outside [1,8]");
    if (n_iv < 0 || (n_iv > 0 && (!iv_lo || !iv_hi)))
        return fail(c, FE_EINVAL, "bad interval set");
    std::vector<int> ilo(iv_lo, iv_lo + n_iv), ihi(iv_hi, iv_hi + n_iv);
    for (int k = 0; k < n_iv; ++k) {
        const int l = ilo[k], h = ihi[k];
        if (l < 0 || l >= h || h >= TICK_LIMIT)
            return fail(c, FE_EINVAL, "interval %d = (%d,%d] invalid", k, l, h);
        if ((int64_t)h * max_level >= TICK_LIMIT)
            return fail(c, FE_EINVAL, "interval %d too wide for max_level", k);
    }
    HIPCHK(c, hipSetDevice(c->device));
    c->stats = fe_stats{};
    hipStream_t s = c->stream;
    StreamInfo si;
    if ((rc = stream_info(c, ids, ticks, (int)n, num_types, si))) return rc;

    std::vector<LevelOut> levels;
    // level 1: a one-node episode occurs at every event of its type
    double t0 = now_ms();
    if ((rc = ensure(c, c->mn, (size_t)num_types * sizeof(int)))) return rc;
    launch_fill(P<int>(c->mn), 0, num_types, s);
    launch_histogram(ids, (int)n, num_types, P<int>(c->mn), s);
    std::vector<int> hist(num_types);
    HIPCHK(c, hipMemcpyAsync(hist.data(), P<int>(c->mn), num_types * sizeof(int),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    {
        LevelOut L1;
        L1.level = 1;
        L1.ncand = num_types;
        L1.nsurv = num_types;
        for (int e = 0; e < num_types; ++e)
            if (hist[e] >= theta) {
                L1.types.push_back(e);
                L1.upper.push_back(hist[e]);
                L1.exact.push_back(hist[e]);
            }
        L1.nfreq = (int64_t)L1.types.size();
        L1.passes = 1;
        if (c->param[FE_PARAM_KEEP_CANDIDATES]) {
            for (int e = 0; e < num_types; ++e) L1.all_types.push_back(e);
            L1.all_upper = hist;
            L1.all_exact = hist;
        }
        L1.gen_ms = 0;
        L1.count_ms = now_ms() - t0;
        levels.push_back(std::move(L1));
    }
    Episodes F;
    F.m = 1;
    for (int e : levels[0].types) F.key.push_back(e);

    for (int level = 2; level <= max_level && F.count() > 0 && n_iv > 0; ++level) {
        t0 = now_ms();
        const bool htile = c->param[FE_PARAM_HOST_TILING] != 0;
        // level >= 3 with device tiling: the join's ranges are searched on
        // the host and the keys written on the device (they never cross PCIe)
        const bool djoin = !htile && level >= 3;
        Episodes C;
        C.key.swap(c->keypool);
        std::vector<int64_t> jfirst, joff;
        size_t M;
        {
            HTimer ht(c, "host_gen");
            if (level == 2) gen_level2(levels[0].types, ilo, ihi, C);
            else if (!djoin) gen_join(F, C);
            else C.m = level;
            M = djoin ? (size_t)gen_join_plan(F, jfirst, joff) : C.count();
        }
        if (M == 0) break;
        if (M >= (size_t)1 << 31 || M * level >= (size_t)1 << 31)
            return fail(c, FE_ENOMEM, "level %d has too many candidates (%zu)", level, M);
        const double gen_ms = now_ms() - t0;
        t0 = now_ms();
        if ((rc = ensure(c, c->mup, 2 * M * sizeof(int)))) return rc;
        if ((rc = ensure(c, c->mex, 2 * M * sizeof(int)))) return rc;
        if ((rc = ensure(c, c->msel, M * sizeof(int)))) return rc;
        if ((rc = ensure(c, c->mn, 4 * sizeof(int)))) return rc;
        int *up = P<int>(c->mup), *ex = P<int>(c->mex);
        // the level's keys go to the device once; tile records are built there
        const int wbound = (level - 1) * *std::max_element(ihi.begin(), ihi.end());
        int bbound = 1;  // largest window bound of the interval set
        for (int k = 0; k < n_iv; ++k) bbound = std::max(bbound, window_bound(ilo[k], ihi[k]));
        const int wk = 3 * level - 2;  // ints per key
        if ((rc = ensure(c, c->mkey, std::max<size_t>(M * wk, 1) * sizeof(int)))) return rc;
        if (djoin) {
            const int64_t cnt = (int64_t)F.count();
            const size_t fb = F.key.size() * sizeof(int), ob = (size_t)(cnt + 1) * sizeof(int64_t);
            if ((rc = ensure(c, c->mfk, fb))) return rc;
            if ((rc = ensure(c, c->mfo, 2 * ob))) return rc;
            HTimer ht(c, "host_upload");
            HIPCHK(c, hipMemcpyAsync(c->mfk.p, F.key.data(), fb, hipMemcpyHostToDevice, s));
            HIPCHK(c, hipMemcpyAsync(c->mfo.p, jfirst.data(), cnt * sizeof(int64_t),
                                     hipMemcpyHostToDevice, s));
            HIPCHK(c, hipMemcpyAsync((char *)c->mfo.p + ob, joff.data(), ob,
                                     hipMemcpyHostToDevice, s));
            launch_join(P<int>(c->mfk), 3 * F.m - 2, (const int64_t *)c->mfo.p,
                        (const int64_t *)((char *)c->mfo.p + ob), cnt, (int64_t)M,
                        P<int>(c->mkey), s);
            HIPCHK(c, hipGetLastError());
            // (F, jfirst and joff outlive the stream synchronisation below)
        } else {
            // (pinned when large: the copy overlaps the host tiling below)
            HTimer ht(c, "host_upload");
            HIPCHK(c, hipMemcpyAsync(P<int>(c->mkey), C.key.data(), C.key.size() * sizeof(int),
                                     hipMemcpyHostToDevice, s));
        }
        HostPack hp;
        ivec order;
        const int64_t emode = c->param[FE_PARAM_ELIMINATION];
        bool elim = emode != 0;
        int64_t smp_n = 0, smp_kept = 0;
        if (emode == 2 && !htile && (int64_t)M >= c->param[FE_PARAM_SAMPLE_MIN]) {
            // two passes pay when the relaxed pass (cost r per candidate,
            // relative to the exact one) prunes more than r of the level;
            // with r >= 1 nothing can, and no sample is taken
            const double r = (double)c->param[FE_PARAM_PASS1_COST] / 1000.0;
            elim = false;
            if (r < 1.0) {
                if ((rc = sample_survival(c, ids, ticks, si, level, (int64_t)M, wbound, bbound,
                                          theta, smp_n, smp_kept)))
                    return rc;
                elim = (double)smp_kept < (1.0 - r) * (double)smp_n;
            }
        }
        int64_t kept = 0;  // candidates of the exact pass (device tiling)
        if (!htile) {
            // prune and tile on the device: pass 1 (Algorithm 3) over every
            // candidate, then pass 2 (Algorithm 1) over those with
            // upper >= theta (Algorithm 4), or over all in one-pass mode
            std::vector<GroupDesc> groups;
            if (elim) {
                if ((rc = dev_pack(c, P<int>(c->mkey), level, (int64_t)M, nullptr, 0, false,
                                   wbound, bbound, groups, kept)))
                    return rc;
                if ((rc = launch_groups(c, ids, ticks, si, groups, false, up))) return rc;
            } else {
                launch_fill(up, -1, (int64_t)M, s);
            }
            launch_fill(ex, -1, (int64_t)M, s);
            if ((rc = dev_pack(c, P<int>(c->mkey), level, (int64_t)M, elim ? up : nullptr, theta,
                               true, wbound, bbound, groups, kept)))
                return rc;
            if (kept > 0 && (rc = launch_groups(c, ids, ticks, si, groups, true, ex))) return rc;
        } else if (elim) {
            // pass 1 (Algorithm 3) over every candidate
            {
                HTimer ht(c, "host_pack");
                host_pack(C, nullptr, (int64_t)M, false, hp, wbound, &c->lanepool);
            }
            {
                HTimer ht(c, "host_upload");
                if ((rc = upload_lanes(c, hp, P<int>(c->mkey), level))) return rc;
            }
            if ((rc = launch_groups(c, ids, ticks, si, hp.groups, false, up))) return rc;
            // elimination (Algorithm 4): survivors have upper >= theta
            ivec uph;
            uph.swap(c->uphpool);
            uph.resize(M);
            order.swap(c->orderpool);
            HIPCHK(c, hipStreamSynchronize(s));
            c->lanepool.swap(hp.orig);  // its upload has completed
            {
                HTimer ht(c, "host_select");
                HIPCHK(c, hipMemcpyAsync(uph.data(), up, M * sizeof(int), hipMemcpyDeviceToHost,
                                         s));
                HIPCHK(c, hipStreamSynchronize(s));
                par_select((int64_t)M, [&](int64_t i) { return uph[i] >= theta; }, order);
            }
            c->uphpool.swap(uph);
        } else {
            // one pass: Algorithm 1 over every candidate, no relaxed count
            launch_fill(up, -1, (int64_t)M, s);
        }
        const int64_t nsurv = !htile ? kept : elim ? (int64_t)order.size() : (int64_t)M;
        // pass 2 (Algorithm 1) over the survivors; the others keep -1
        if (htile) launch_fill(ex, -1, (int64_t)M, s);
        if (htile && nsurv > 0) {
            {
                HTimer ht(c, "host_pack");
                host_pack(C, elim ? order.data() : nullptr, nsurv, true, hp, wbound,
                          &c->lanepool);
            }
            {
                HTimer ht(c, "host_upload");
                if ((rc = upload_lanes(c, hp, P<int>(c->mkey), level))) return rc;
            }
            if ((rc = launch_groups(c, ids, ticks, si, hp.groups, true, ex))) return rc;
        }
        // frequent = exact >= theta
        launch_fill(P<int>(c->mn), 0, 1, s);
        launch_compact(ex, (int)M, theta, nullptr, P<int>(c->msel), P<int>(c->mn), s);
        launch_gather2(up, ex, P<int>(c->msel), P<int>(c->mn), (int)M, up + M, ex + M, s);
        int cnts[2];
        HIPCHK(c, hipMemcpyAsync(cnts, P<int>(c->mn), sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        cnts[1] = (int)nsurv;
        const int nf = cnts[0];
        std::vector<int> fsel(nf), fup(nf), fex(nf);
        if (nf > 0) {
            HIPCHK(c, hipMemcpyAsync(fsel.data(), P<int>(c->msel), nf * sizeof(int),
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipMemcpyAsync(fup.data(), up + M, nf * sizeof(int), hipMemcpyDeviceToHost,
                                     s));
            HIPCHK(c, hipMemcpyAsync(fex.data(), ex + M, nf * sizeof(int), hipMemcpyDeviceToHost,
                                     s));
            HIPCHK(c, hipStreamSynchronize(s));
        }
        LevelOut Lv;
        Lv.passes = elim ? 2 : 1;
        Lv.sample_n = smp_n;
        Lv.sample_kept = smp_kept;
        if (c->param[FE_PARAM_KEEP_CANDIDATES]) {
            Lv.all_upper.resize(M);
            Lv.all_exact.resize(M);
            HIPCHK(c, hipMemcpyAsync(Lv.all_upper.data(), up, M * sizeof(int),
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipMemcpyAsync(Lv.all_exact.data(), ex, M * sizeof(int),
                                     hipMemcpyDeviceToHost, s));
            std::vector<int> keys;
            const int *kp = C.key.data();
            if (djoin) {
                keys.resize(M * wk);
                HIPCHK(c, hipMemcpyAsync(keys.data(), P<int>(c->mkey), M * wk * sizeof(int),
                                         hipMemcpyDeviceToHost, s));
                kp = keys.data();
            }
            HIPCHK(c, hipStreamSynchronize(s));
            split_keys(kp, M, level, Lv.all_types, Lv.all_lo, Lv.all_hi);
        }
        Episodes NF;
        NF.m = level;
        NF.key.resize((size_t)nf * wk);
        if (djoin) {
            // the frequent keys come back from the device
            if (nf > 0) {
                if ((rc = ensure(c, c->mfsel, (size_t)nf * wk * sizeof(int)))) return rc;
                launch_gather_keys(P<int>(c->mkey), wk, P<int>(c->msel), nf, P<int>(c->mfsel), s);
                HIPCHK(c, hipMemcpyAsync(NF.key.data(), c->mfsel.p, (size_t)nf * wk * sizeof(int),
                                         hipMemcpyDeviceToHost, s));
                HIPCHK(c, hipStreamSynchronize(s));
            }
        } else {
            for (int i = 0; i < nf; ++i)
                std::memcpy(NF.key.data() + (size_t)i * wk, C.at(fsel[i]), wk * sizeof(int));
        }
        {
            HTimer ht(c, "host_sort");
            // (the join writes candidates in key order; the compaction that
            // found the frequent ones does not keep it)
            if (djoin) order_by_index(NF, fsel, (int64_t)M, &fup, &fex);
            else sort_episodes(NF, &fup, &fex);
        }
        Lv.level = level;
        Lv.ncand = (int64_t)M;
        Lv.nsurv = cnts[1];
        Lv.nfreq = nf;
        Lv.types.resize((size_t)nf * level);
        Lv.lo.resize((size_t)nf * (level - 1));
        Lv.hi.resize((size_t)nf * (level - 1));
        for (int i = 0; i < nf; ++i) {
            const int *k = NF.at(i);
            for (int j = 0; j < level; ++j) Lv.types[(size_t)i * level + j] = k[3 * j];
            for (int j = 0; j < level - 1; ++j) {
                Lv.lo[(size_t)i * (level - 1) + j] = k[3 * j + 1];
                Lv.hi[(size_t)i * (level - 1) + j] = k[3 * j + 2];
            }
        }
        Lv.upper = fup;
        Lv.exact = fex;
        Lv.gen_ms = gen_ms;
        Lv.count_ms = now_ms() - t0;
        levels.push_back(std::move(Lv));
        F.m = level;
        F.key.swap(NF.key);
        // (their copies to the device have completed: synchronised above)
        c->keypool.swap(C.key);
        if (hp.orig.capacity() > c->lanepool.capacity()) c->lanepool.swap(hp.orig);
        c->orderpool.swap(order);
    }

    fe_result *r = (fe_result *)std::calloc(1, sizeof(fe_result));
    if (!r) return fail(c, FE_ENOMEM, "host allocation failed");
    r->n_levels = (int)levels.size();
    r->levels = (fe_level *)std::calloc(levels.size(), sizeof(fe_level));
    if (!r->levels) {
        std::free(r);
        return fail(c, FE_ENOMEM, "host allocation failed");
    }
    auto dup = [](const std::vector<int> &v) {
        int *p = (int *)std::malloc(std::max<size_t>(v.size(), 1) * sizeof(int));
        if (p && !v.empty()) std::memcpy(p, v.data(), v.size() * sizeof(int));
        return p;
    };
    for (size_t i = 0; i < levels.size(); ++i) {
        fe_level &d = r->levels[i];
        const LevelOut &L = levels[i];
        d.level = L.level;
        d.n_candidates = L.ncand;
        d.n_survivors = L.nsurv;
        d.n_frequent = L.nfreq;
        d.types = dup(L.types);
        d.lo = dup(L.lo);
        d.hi = dup(L.hi);
        d.upper = dup(L.upper);
        d.exact = dup(L.exact);
        d.gen_ms = L.gen_ms;
        d.count_ms = L.count_ms;
        d.passes = L.passes;
        d.sample_n = L.sample_n;
        d.sample_kept = L.sample_kept;
        auto dup_opt = [&](const std::vector<int> &v, bool on) { return on ? dup(v) : nullptr; };
        const bool all = !L.all_exact.empty() || (L.ncand == 0 && c->param[FE_PARAM_KEEP_CANDIDATES]);
        d.all_types = dup_opt(L.all_types, all);
        d.all_lo = dup_opt(L.all_lo, all);
        d.all_hi = dup_opt(L.all_hi, all);
        d.all_upper = dup_opt(L.all_upper, all);
        d.all_exact = dup_opt(L.all_exact, all);
    }
    *out = r;
    c->stats.last_call_ms = now_ms() - t_call;
    return FE_OK;
}

extern "C" void fe_result_free(fe_result *r)
{
    if (!r) return;
    for (int i = 0; i < r->n_levels; ++i) {
        std::free(r->levels[i].types);
        std::free(r->levels[i].lo);
        std::free(r->levels[i].hi);
        std::free(r->levels[i].upper);
        std::free(r->levels[i].exact);
        std::free(r->levels[i].all_types);
        std::free(r->levels[i].all_lo);
        std::free(r->levels[i].all_hi);
        std::free(r->levels[i].all_upper);
        std::free(r->levels[i].all_exact);
    }
    std::free(r->levels);
    std::free(r);
}

// ====================================================================== batching

struct fe_batch {
    fe_ctx *c = nullptr;
    std::vector<fe_job> jobs;
    std::vector<StreamInfo> si;
    // tiling (independent of the launch shape)
    struct Group {
        int job, key, t0, tiles, wmax, dcap;
    };
    std::vector<Group> groups;
    std::vector<int> rec, orig, tileW;
    int ntiles = 0;
    fe_batch_tuning tun{32768, 16, WPB, 0.0};
    // device
    Buf pk, origd, tileWd, tilesd, jobsd, itemsd, listsd, lamd, tbld, flagsr, flagsx, qctr, deepd;
    struct Level {
        int N;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
    };
    std::vector<Level> levels;
    hipStream_t cap = nullptr;
    int ncu = 256;
};

namespace {

void batch_free_graphs(fe_batch *b)
{
    for (auto &L : b->levels) {
        if (L.x) (void)hipGraphExecDestroy(L.x);
        if (L.g) (void)hipGraphDestroy(L.g);
    }
    b->levels.clear();
}

int batch_P(const fe_ctx *c, int n, int span, int wmax, int seg_events)
{
    if (n <= 1) return 1;
    const double lb = (double)n * (double)wmax / std::max(span, 1);
    const int64_t minseg = std::max<int64_t>(c->param[FE_PARAM_MIN_SEG_EVENTS],
                                             (int64_t)(8.0 * lb) + 64);
    int64_t P = (n + (int64_t)seg_events - 1) / std::max(seg_events, 1);
    P = std::min<int64_t>(P, std::max<int64_t>(1, n / minseg));
    return (int)std::max<int64_t>(1, std::min<int64_t>(P, 256));
}

// Launch plan for the current tuning: per-tile descriptors, work items,
// tile lists, device buffers and one captured graph per episode size.
int batch_plan(fe_batch *b)
{
    fe_ctx *c = b->c;
    int rc;
    batch_free_graphs(b);
    const int T = b->ntiles;
    std::vector<TileDesc> td(T);
    std::vector<int> tileN(T), tileD(T);
    int64_t lam_off = 0, tbl_off = 0;
    for (const auto &g : b->groups) {
        const StreamInfo &si = b->si[g.job];
        const int P = batch_P(c, si.n, si.span, g.wmax, b->tun.seg_events);
        for (int t = g.t0; t < g.t0 + g.tiles; ++t) {
            td[t].job = g.job;
            td[t].P = P;
            td[t].otile = t;
            td[t].rec = 0;
            td[t].lam = lam_off;
            td[t].tbl = tbl_off;
            tileN[t] = g.key / NDCLS + 1;
            tileD[t] = g.key % NDCLS;
            if (P > 1) {
                lam_off += P + 1;
                tbl_off += (int64_t)P * WAVE * KMAX;
            }
        }
    }
    // record offsets follow the packed order
    {
        int64_t off = 0;
        for (const auto &g : b->groups) {
            const int N = g.key / NDCLS + 1;
            for (int t = g.t0; t < g.t0 + g.tiles; ++t) {
                td[t].rec = off;
                off += rec_ints(N);
            }
        }
    }
    // items and tile lists per level
    std::vector<int2> items;
    std::vector<int> lists;
    struct LvPlan {
        int N;
        int64_t it_rel, n_rel;
        int64_t it_ex[NDCLS], n_ex[NDCLS];
        int64_t pl, npl;                   // P > 1 tiles of the level
        int64_t pld[NDCLS], npld[NDCLS];   // P > 1 tiles per depth class
    };
    std::vector<LvPlan> lp;
    for (int N = 1; N <= NMAX; ++N) {
        std::vector<int> tl;
        for (int t = 0; t < T; ++t)
            if (tileN[t] == N) tl.push_back(t);
        if (tl.empty()) continue;
        LvPlan L{};
        L.N = N;
        auto add_items = [&](const std::vector<int> &ts, int64_t &off, int64_t &cnt) {
            std::vector<std::pair<int64_t, int2>> v;
            for (int t : ts) {
                const int P = td[t].P;
                const int64_t cost = (int64_t)b->si[td[t].job].n / P;
                for (int p = 0; p < P; ++p) v.push_back({cost, make_int2(t, p)});
            }
            std::stable_sort(v.begin(), v.end(),
                             [](const std::pair<int64_t, int2> &a,
                                const std::pair<int64_t, int2> &bb) { return a.first > bb.first; });
            off = (int64_t)items.size();
            cnt = (int64_t)v.size();
            for (auto &e : v) items.push_back(e.second);
        };
        add_items(tl, L.it_rel, L.n_rel);
        for (int d = 0; d < NDCLS; ++d) {
            if (d == DEEP_CLS) continue;  // counted by k_deep, whole stream
            std::vector<int> td_d;
            for (int t : tl)
                if (tileD[t] == d) td_d.push_back(t);
            add_items(td_d, L.it_ex[d], L.n_ex[d]);
            L.pld[d] = (int64_t)lists.size();
            for (int t : td_d)
                if (td[t].P > 1) lists.push_back(t);
            L.npld[d] = (int64_t)lists.size() - L.pld[d];
        }
        L.pl = (int64_t)lists.size();
        for (int t : tl)
            if (td[t].P > 1) lists.push_back(t);
        L.npl = (int64_t)lists.size() - L.pl;
        lp.push_back(L);
    }
    std::vector<BJob> bj(b->jobs.size());
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        bj[j].ids = b->jobs[j].ids;
        bj[j].ticks = b->jobs[j].ticks;
        bj[j].n = (int)b->jobs[j].n;
        bj[j].theta = b->jobs[j].theta;
        bj[j].upper = b->jobs[j].upper_out;
        bj[j].exact = b->jobs[j].exact_out;
    }
    // deep-class groups: the exact pass by k_deep over the recording's stream
    struct DeepJob {
        int N, job, t0, tiles;
        DeepPlan dp;
    };
    std::vector<DeepJob> dj;
    int64_t deep_bytes = 0;
    for (const auto &g : b->groups) {
        if (g.key % NDCLS != DEEP_CLS) continue;
        const int N = g.key / NDCLS + 1;
        const DeepPlan dp = deep_plan(N, (int64_t)g.tiles * WAVE, g.dcap, (int)b->jobs[g.job].n);
        deep_bytes = std::max(deep_bytes, dp.bytes);
        dj.push_back(DeepJob{N, g.job, g.t0, g.tiles, dp});
    }
    hipStream_t s = c->stream;
    HIPCHK(c, hipStreamSynchronize(s));
    if (deep_bytes > 0 && (rc = ensure(c, b->deepd, (size_t)deep_bytes))) return rc;
    if ((rc = ensure(c, b->tilesd, std::max<size_t>(td.size(), 1) * sizeof(TileDesc)))) return rc;
    if ((rc = ensure(c, b->jobsd, std::max<size_t>(bj.size(), 1) * sizeof(BJob)))) return rc;
    if ((rc = ensure(c, b->itemsd, std::max<size_t>(items.size(), 1) * sizeof(int2)))) return rc;
    if ((rc = ensure(c, b->listsd, std::max<size_t>(lists.size(), 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, b->lamd, std::max<int64_t>(lam_off, 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, b->tbld, std::max<int64_t>(tbl_off, 1) * sizeof(int2)))) return rc;
    if ((rc = ensure(c, b->flagsr, std::max<int64_t>((int64_t)T * WAVE, 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, b->flagsx, std::max<int64_t>((int64_t)T * WAVE, 1) * sizeof(int)))) return rc;
    if ((rc = ensure(c, b->qctr, (size_t)(NMAX * (1 + NDCLS)) * sizeof(int)))) return rc;
    HIPCHK(c, hipMemcpy(b->tilesd.p, td.data(), td.size() * sizeof(TileDesc), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(b->jobsd.p, bj.data(), bj.size() * sizeof(BJob), hipMemcpyHostToDevice));
    if (!items.empty())
        HIPCHK(c, hipMemcpy(b->itemsd.p, items.data(), items.size() * sizeof(int2),
                            hipMemcpyHostToDevice));
    if (!lists.empty())
        HIPCHK(c, hipMemcpy(b->listsd.p, lists.data(), lists.size() * sizeof(int),
                            hipMemcpyHostToDevice));
    launch_fill(P<int>(b->flagsr), 0, (int64_t)T * WAVE, s);
    launch_fill(P<int>(b->flagsx), 0, (int64_t)T * WAVE, s);
    HIPCHK(c, hipStreamSynchronize(s));

    const int grid = std::max(1, b->ncu * b->tun.waves_per_cu / b->tun.waves_per_block);
    int *lists_d = P<int>(b->listsd);
    int q = 0;
    for (const LvPlan &L : lp) {
        fe_batch::Level lv;
        lv.N = L.N;
        HIPCHK(c, hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        hipStream_t cs = b->cap;
        BatchDev d;
        d.tiles = (const TileDesc *)b->tilesd.p;
        d.jobs = (const BJob *)b->jobsd.p;
        d.pk = P<int>(b->pk);
        d.orig = P<int>(b->origd);
        d.lam = P<int>(b->lamd);
        d.tbl = P<int2>(b->tbld);
        d.status = P<int>(c->status);
        d.sparse = c->param[FE_PARAM_TYPE_DISPATCH] != 0;
        d.wpb = b->tun.waves_per_block;
        const int q0 = q;
        int nq = 1;
        for (int dd = 0; dd < NDCLS; ++dd) nq += L.n_ex[dd] > 0;
        launch_fill(P<int>(b->qctr) + q0, 0, nq, cs);
        launch_clear_flags(lists_d + L.pl, (int)L.npl, P<int>(b->flagsr), P<int>(b->flagsx), cs);
        launch_plan_batch(d.tiles, d.jobs, P<int>(b->tileWd), lists_d + L.pl, (int)L.npl,
                          P<int>(b->lamd), cs);
        // pass 1: relaxed, every candidate of this size
        d.items = P<int2>(b->itemsd) + L.it_rel;
        d.nitems = (int)L.n_rel;
        d.qctr = P<int>(b->qctr) + q++;
        d.flags = P<int>(b->flagsr);
        launch_persist(L.N, false, 0, d, grid, cs);
        launch_concat_batch(d, lists_d + L.pl, (int)L.npl, false, cs);
        launch_persist_fixup(L.N, false, 0, d, lists_d + L.pl, (int)L.npl, cs);
        // pass 2: exact, survivors only
        d.flags = P<int>(b->flagsx);
        for (int dd = 0; dd < NDCLS; ++dd) {
            if (!L.n_ex[dd]) continue;
            d.items = P<int2>(b->itemsd) + L.it_ex[dd];
            d.nitems = (int)L.n_ex[dd];
            d.qctr = P<int>(b->qctr) + q++;
            launch_persist(L.N, true, dd, d, grid, cs);
        }
        for (int dd = 0; dd < NDCLS; ++dd)
            if (L.npld[dd]) {
                launch_concat_batch(d, lists_d + L.pld[dd], (int)L.npld[dd], true, cs);
                launch_persist_fixup(L.N, true, dd, d, lists_d + L.pld[dd], (int)L.npld[dd], cs);
            }
        for (const DeepJob &x : dj) {
            if (x.N != L.N) continue;
            const fe_job &j = b->jobs[x.job];
            DeepArgs a{};
            a.ids = j.ids;
            a.ticks = j.ticks;
            a.n = (int)j.n;
            a.pk = P<int>(b->pk) + td[x.t0].rec;
            a.orig = P<int>(b->origd) + (int64_t)x.t0 * WAVE;
            a.ring = P<int2>(b->deepd);
            a.out = j.exact_out;
            a.upper = j.upper_out;
            a.theta = j.theta;
            a.status = P<int>(c->status);
            deep_launch(x.N, a, x.dp, (int64_t)x.tiles * WAVE, cs);
        }
        hipError_t e1 = hipStreamEndCapture(b->cap, &lv.g);
        if (e1 != hipSuccess) return fail(c, FE_EDEVICE, "graph capture failed: %s", hipGetErrorString(e1));
        HIPCHK(c, hipGraphInstantiate(&lv.x, lv.g, nullptr, nullptr, 0));
        b->levels.push_back(lv);
        (void)q0;
    }
    return FE_OK;
}

}  // namespace

extern "C" int fe_batch_create(fe_ctx *c, int32_t R, const fe_job *jobs, fe_batch **out)
{
    int rc;
    if (!c || !out) return FE_EINVAL;
    *out = nullptr;
    if (R < 0 || (R > 0 && !jobs)) return fail(c, FE_EINVAL, "bad job list");
    for (int r = 0; r < R; ++r) {
        const fe_job &j = jobs[r];
        if ((rc = check_common(c, j.ids, j.ticks, j.n, j.num_types))) return rc;
        if ((rc = check_cands(c, j.types, j.len, j.lo, j.hi, j.M, j.nmax))) return rc;
        if (j.M > 0 && (!j.upper_out || !j.exact_out))
            return fail(c, FE_EINVAL, "job %d: null output", r);
    }
    HIPCHK(c, hipSetDevice(c->device));
    fe_batch *b = new (std::nothrow) fe_batch();
    if (!b) return fail(c, FE_ENOMEM, "host allocation failed");
    b->c = c;
    b->jobs.assign(jobs, jobs + R);
    b->si.resize(R);
    (void)hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(c, FE_EDEVICE, "stream creation failed");
    }
    auto bail = [&](int code) {
        fe_batch_destroy(b);
        return code;
    };
    // validate the streams and learn their spans
    for (int r = 0; r < R; ++r)
        if ((rc = stream_info(c, jobs[r].ids, jobs[r].ticks, (int)jobs[r].n, jobs[r].num_types,
                              b->si[r])))
            return bail(rc);
    // candidate tables to the host, checked, tiled per episode size
    int64_t rec_total = 0;
    for (int r = 0; r < R; ++r) {
        const fe_job &j = jobs[r];
        if (j.M == 0) continue;
        const int nm = j.nmax, hm = std::max(nm - 1, 1);
        std::vector<int> ty((size_t)j.M * nm), ln(j.M), lo((size_t)j.M * hm), hi((size_t)j.M * hm);
        HIPCHK(c, hipMemcpy(ty.data(), j.types, ty.size() * sizeof(int), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(ln.data(), j.len, ln.size() * sizeof(int), hipMemcpyDeviceToHost));
        if (nm > 1) {
            HIPCHK(c, hipMemcpy(lo.data(), j.lo, (size_t)j.M * (nm - 1) * sizeof(int),
                                hipMemcpyDeviceToHost));
            HIPCHK(c, hipMemcpy(hi.data(), j.hi, (size_t)j.M * (nm - 1) * sizeof(int),
                                hipMemcpyDeviceToHost));
        }
        for (int N = 1; N <= nm; ++N) {
            Episodes C;
            C.m = N;
            std::vector<int> back;
            for (int m = 0; m < j.M; ++m) {
                const int L = ln[m];
                if (L < 1 || L > nm) return bail(fail(c, FE_EINVAL, "job %d: bad len", r));
                if (L != N) continue;
                int64_t W = 0;
                for (int k = 0; k < N; ++k) {
                    const int t = ty[(size_t)m * nm + k];
                    if (t < 0 || t >= j.num_types)
                        return bail(fail(c, FE_EINVAL, "job %d: type out of range", r));
                    C.key.push_back(t);
                    if (k < N - 1) {
                        const int l = lo[(size_t)m * (nm - 1) + k], h = hi[(size_t)m * (nm - 1) + k];
                        if (l < 0 || l >= h || h >= TICK_LIMIT)
                            return bail(fail(c, FE_EINVAL, "job %d: bad interval", r));
                        W += h;
                        C.key.push_back(l);
                        C.key.push_back(h);
                    }
                }
                if (W >= TICK_LIMIT) return bail(fail(c, FE_EINVAL, "job %d: W too large", r));
                back.push_back(m);
            }
            if (back.empty()) continue;
            HostPack hp;
            host_pack(C, nullptr, (int64_t)back.size(), true, hp);
            for (const GroupDesc &gd : hp.groups) {
                fe_batch::Group g{r, gd.key, b->ntiles + gd.tile_base, gd.tiles, gd.wmax,
                                  gd.dcap};
                b->groups.push_back(g);
            }
            b->rec.insert(b->rec.end(), hp.rec.begin(), hp.rec.end());
            for (int o : hp.orig) b->orig.push_back(o < 0 ? -1 : back[o]);
            b->tileW.insert(b->tileW.end(), hp.tileW.begin(), hp.tileW.end());
            b->ntiles += hp.tiles;
            rec_total += (int64_t)hp.rec.size();
        }
    }
    if ((rc = ensure(c, b->pk, std::max<int64_t>(rec_total, 1) * sizeof(int)))) return bail(rc);
    if ((rc = ensure(c, b->origd, std::max<size_t>(b->orig.size(), 1) * sizeof(int)))) return bail(rc);
    if ((rc = ensure(c, b->tileWd, std::max<size_t>(b->tileW.size(), 1) * sizeof(int)))) return bail(rc);
    if (!b->rec.empty())
        HIPCHK(c, hipMemcpy(b->pk.p, b->rec.data(), b->rec.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!b->orig.empty())
        HIPCHK(c, hipMemcpy(b->origd.p, b->orig.data(), b->orig.size() * sizeof(int),
                            hipMemcpyHostToDevice));
    if (!b->tileW.empty())
        HIPCHK(c, hipMemcpy(b->tileWd.p, b->tileW.data(), b->tileW.size() * sizeof(int),
                            hipMemcpyHostToDevice));
    b->rec.clear();
    b->rec.shrink_to_fit();
    if ((rc = batch_plan(b))) return bail(rc);
    *out = b;
    return FE_OK;
}

extern "C" int fe_batch_run(fe_batch *b)
{
    if (!b) return FE_EINVAL;
    fe_ctx *c = b->c;
    HIPCHK(c, hipSetDevice(c->device));
    for (auto &L : b->levels) HIPCHK(c, hipGraphLaunch(L.x, c->stream));
    return FE_OK;
}

extern "C" int fe_batch_set_tuning(fe_batch *b, const fe_batch_tuning *t)
{
    const int wpb = t ? (t->waves_per_block ? t->waves_per_block : WPB) : 0;
    if (!b || !t || t->seg_events < 256 || t->waves_per_cu < 1 || t->waves_per_cu > 64 ||
        wpb < 1 || wpb > PERSIST_WPB_MAX || (wpb & (wpb - 1)))
        return FE_EINVAL;
    b->tun.seg_events = t->seg_events;
    b->tun.waves_per_cu = t->waves_per_cu;
    b->tun.waves_per_block = wpb;
    return batch_plan(b);
}

extern "C" int fe_batch_get_tuning(const fe_batch *b, fe_batch_tuning *t)
{
    if (!b || !t) return FE_EINVAL;
    *t = b->tun;
    return FE_OK;
}

extern "C" int fe_batch_autotune(fe_batch *b, int32_t reps, fe_batch_tuning *best)
{
    if (!b || reps < 1) return FE_EINVAL;
    fe_ctx *c = b->c;
    int rc;
    const int segs[] = {8192, 16384, 32768, 65536, 131072};
    const int wpcs[] = {8, 16, 32};
    const int wpbs[] = {2, 4, 8};
    fe_batch_tuning top{0, 0, 0, 1e30};
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    for (int sg : segs)
        for (int wp : wpcs)
        for (int wb : wpbs) {
            b->tun.seg_events = sg;
            b->tun.waves_per_cu = wp;
            b->tun.waves_per_block = wb;
            if ((rc = batch_plan(b))) return rc;
            if ((rc = fe_batch_run(b))) return rc;  // warm-up
            HIPCHK(c, hipEventRecord(e0, c->stream));
            for (int r = 0; r < reps; ++r)
                if ((rc = fe_batch_run(b))) return rc;
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            if (ms / reps < top.run_ms) top = fe_batch_tuning{sg, wp, wb, ms / reps};
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tun = top;
    if ((rc = batch_plan(b))) return rc;
    if (best) *best = top;
    return FE_OK;
}

extern "C" int fe_batch_destroy(fe_batch *b)
{
    if (!b) return FE_EINVAL;
    fe_ctx *c = b->c;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    batch_free_graphs(b);
    Buf *bufs[] = {&b->pk,    &b->origd, &b->tileWd, &b->tilesd, &b->jobsd,  &b->itemsd,
                   &b->listsd, &b->lamd, &b->tbld,   &b->flagsr, &b->flagsx, &b->qctr,
                   &b->deepd};
    for (Buf *x : bufs)
        if (x->p) (void)hipFree(x->p);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return FE_OK;
}

extern "C" int fe_count_batched(fe_ctx *c, int32_t R, const fe_job *jobs)
{
    fe_batch *b = nullptr;
    int rc = fe_batch_create(c, R, jobs, &b);
    if (rc) return rc;
    rc = fe_batch_run(b);
    if (!rc) rc = fe_sync(c);
    fe_batch_destroy(b);
    return rc;
}

// ====================================================================== serving

namespace {

int64_t steady_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

struct fe_server {
    fe_ctx *c = nullptr;
    fe_server_config cfg{};
    int M = 0;
    // resident candidates, packed once
    Buf pk, origd, tileWd;
    std::vector<GroupDesc> groups;
    std::vector<int64_t> tile_rec;  // record offset per packed tile
    std::vector<int> tile_key;      // group key per packed tile
    std::vector<int> tile_w;        // widest W per packed tile
    int ntiles = 0;
    // arrays
    struct Arr {
        Buf ids, ticks;
        std::vector<int> hticks;  // host mirror of the ticks (request windows)
        int64_t n = 0;
        int num_types = 0;
    };
    std::vector<Arr> arr;
    std::mutex amu;  // guards appends against window lookups
    // appends: asynchronous copies from a pinned staging ring on a stream of
    // their own; every round waits for the last one (aev) before it starts
    hipStream_t astream = nullptr;
    hipEvent_t aev = nullptr;
    char *astage = nullptr;
    size_t astage_cap = 0, apos = 0;
    bool apending = false;
    // requests
    struct Req {
        fe_request r;
        uint64_t ticket;
        int a = 0, b = 0;  // event index range of the window
        int status = FE_OK;
        int state = 0;     // 0 queued, 1 running, 2 done
        int64_t arrival = 0, admit = 0, done = 0;
        int round = -1, rsize = 0;
        int ns = 0, nf = 0;
        int64_t foot = 0;
        std::vector<int> up, ex;
    };
    std::unordered_map<uint64_t, Req *> reqs;
    std::deque<Req *> pending;
    uint64_t next_ticket = 1;
    // device lanes: one stream and one arena each
    struct Lane {
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
        bool busy = false;
        std::vector<Req *> reqs;
        Buf arena, outd, descd, jobsd;
        Buf statd;               // device status word of the lane's rounds
        Buf deepd;               // window rings of deep-class candidates
        int *hout = nullptr;     // pinned results, then the round's status word
        char *hstage = nullptr;  // pinned staging for descriptors and items
        size_t stage_cap = 0;
    };
    std::vector<Lane> lanes;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    fe_server_stats st{};
    int round_id = 0;
    int ncu = 256;
};

namespace {

// Device state one request needs inside a lane's arena (slot tables, look-
// back starts, flags, work items, tile lists).
int64_t req_arena_bytes(const fe_server *sv, int n)
{
    int64_t tot = 0;
    for (const GroupDesc &g : sv->groups) {
        const int P = std::max(1, (int)std::min<int64_t>(256, (n + sv->cfg.seg_events - 1) /
                                                             std::max(1, sv->cfg.seg_events)));
        tot += (int64_t)g.tiles * (P > 1 ? ((int64_t)P * WAVE * KMAX * 8 + (P + 1) * 4 + 4) : 0);
        tot += (int64_t)g.tiles * P * 8;          // items
        tot += (int64_t)g.tiles * WAVE * 4 * 2;   // flags
    }
    return tot + 4096;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Plan and enqueue one round on a lane.
int server_launch(fe_server *sv, fe_server::Lane &ln)
{
    fe_ctx *c = sv->c;
    const int R = (int)ln.reqs.size();
    const int T = sv->ntiles;
    const int M = sv->M;
    std::vector<TileDesc> td;
    td.reserve((size_t)R * T);
    std::vector<BJob> bj(R);
    std::vector<int> descN, descD;
    int64_t lam_off = 0, tbl_off = 0;
    for (int r = 0; r < R; ++r) {
        fe_server::Req *q = ln.reqs[r];
        const fe_server::Arr &A = sv->arr[q->r.array];
        const int n = q->b - q->a;
        const int span = n > 0 ? A.hticks[q->b - 1] - A.hticks[q->a] + 1 : 1;
        bj[r].ids = P<int>(const_cast<Buf &>(A.ids)) + q->a;
        bj[r].ticks = P<int>(const_cast<Buf &>(A.ticks)) + q->a;
        bj[r].n = n;
        bj[r].theta = q->r.theta;
        bj[r].upper = P<int>(ln.outd) + (int64_t)r * 2 * M;
        bj[r].exact = P<int>(ln.outd) + (int64_t)r * 2 * M + M;
        for (const GroupDesc &g : sv->groups) {
            const int Pn = batch_P(c, n, span, g.wmax, sv->cfg.seg_events);
            for (int t = g.tile_base; t < g.tile_base + g.tiles; ++t) {
                TileDesc d;
                d.job = r;
                d.P = Pn;
                d.otile = t;
                d.rec = sv->tile_rec[t];
                d.lam = lam_off;
                d.tbl = tbl_off;
                if (Pn > 1) {
                    lam_off += Pn + 1;
                    tbl_off += (int64_t)Pn * WAVE * KMAX;
                }
                td.push_back(d);
                descN.push_back(g.key / NDCLS + 1);
                descD.push_back(g.key % NDCLS);
            }
        }
    }
    const int D = (int)td.size();
    // work items and tile lists per episode size
    std::vector<int2> items;
    std::vector<int> lists;
    struct LvPlan {
        int N;
        int64_t it_rel, n_rel, it_ex[NDCLS], n_ex[NDCLS], pl, npl, pld[NDCLS], npld[NDCLS];
    };
    std::vector<LvPlan> lp;
    for (int N = 1; N <= NMAX; ++N) {
        std::vector<int> tl;
        for (int t = 0; t < D; ++t)
            if (descN[t] == N) tl.push_back(t);
        if (tl.empty()) continue;
        LvPlan L{};
        L.N = N;
        // work items heaviest first (cost n/P); the tiles of one request and
        // group share their cost, so runs of equal-cost tiles are ordered,
        // not the items one by one
        auto add_items = [&](const std::vector<int> &ts, int64_t &off, int64_t &cnt) {
            std::vector<std::pair<int64_t, size_t>> runs;  // (cost, first position in ts)
            for (size_t i = 0; i < ts.size(); ++i) {
                const int t = ts[i];
                const int64_t cost = (int64_t)bj[td[t].job].n / td[t].P + 1;
                if (i == 0 || td[t].job != td[ts[i - 1]].job || cost != runs.back().first)
                    runs.push_back({cost, i});
            }
            std::stable_sort(runs.begin(), runs.end(),
                             [](const std::pair<int64_t, size_t> &a,
                                const std::pair<int64_t, size_t> &b2) { return a.first > b2.first; });
            off = (int64_t)items.size();
            for (size_t k = 0; k < runs.size(); ++k) {
                const size_t i0 = runs[k].second;
                size_t i1 = i0 + 1;
                while (i1 < ts.size() && td[ts[i1]].job == td[ts[i0]].job &&
                       (int64_t)bj[td[ts[i1]].job].n / td[ts[i1]].P + 1 == runs[k].first)
                    ++i1;
                for (size_t i = i0; i < i1; ++i)
                    for (int p = 0; p < td[ts[i]].P; ++p) items.push_back(make_int2(ts[i], p));
            }
            cnt = (int64_t)items.size() - off;
        };
        add_items(tl, L.it_rel, L.n_rel);
        for (int d = 0; d < NDCLS; ++d) {
            if (d == DEEP_CLS) continue;  // counted by k_deep, whole stream
            std::vector<int> tdd;
            for (int t : tl)
                if (descD[t] == d) tdd.push_back(t);
            add_items(tdd, L.it_ex[d], L.n_ex[d]);
            L.pld[d] = (int64_t)lists.size();
            for (int t : tdd)
                if (td[t].P > 1) lists.push_back(t);
            L.npld[d] = (int64_t)lists.size() - L.pld[d];
        }
        L.pl = (int64_t)lists.size();
        for (int t : tl)
            if (td[t].P > 1) lists.push_back(t);
        L.npl = (int64_t)lists.size() - L.pl;
        lp.push_back(L);
    }
    // carve the lane arena
    size_t off = 0;
    const size_t o_items = off;
    off = align_up(off + std::max<size_t>(items.size(), 1) * sizeof(int2));
    const size_t o_lists = off;
    off = align_up(off + std::max<size_t>(lists.size(), 1) * sizeof(int));
    const size_t o_lam = off;
    off = align_up(off + std::max<int64_t>(lam_off, 1) * sizeof(int));
    const size_t o_tbl = off;
    off = align_up(off + std::max<int64_t>(tbl_off, 1) * sizeof(int2));
    const size_t o_fr = off;
    off = align_up(off + (size_t)D * WAVE * sizeof(int));
    const size_t o_fx = off;
    off = align_up(off + (size_t)D * WAVE * sizeof(int));
    const size_t o_q = off;
    off = align_up(off + NMAX * (1 + NDCLS) * sizeof(int));
    if (off > ln.arena.cap) return fail(c, FE_EINTERNAL, "round exceeds its lane arena");
    char *ar = (char *)ln.arena.p;
    // staging (pinned): descriptors, jobs, items, lists
    const size_t sd = align_up(td.size() * sizeof(TileDesc));
    const size_t sj = align_up(bj.size() * sizeof(BJob));
    const size_t si = align_up(items.size() * sizeof(int2));
    const size_t sl = align_up(lists.size() * sizeof(int));
    const size_t need = sd + sj + si + sl + 1024;
    if (need > ln.stage_cap) {
        if (ln.hstage) HIPCHK(c, hipHostFree(ln.hstage));
        ln.hstage = nullptr;
        HIPCHK(c, hipHostMalloc((void **)&ln.hstage, need * 2));
        ln.stage_cap = need * 2;
    }
    if (td.size() * sizeof(TileDesc) > ln.descd.cap || bj.size() * sizeof(BJob) > ln.jobsd.cap)
        return fail(c, FE_EINTERNAL, "round exceeds its descriptor space");
    std::memcpy(ln.hstage, td.data(), td.size() * sizeof(TileDesc));
    std::memcpy(ln.hstage + sd, bj.data(), bj.size() * sizeof(BJob));
    if (!items.empty()) std::memcpy(ln.hstage + sd + sj, items.data(), items.size() * sizeof(int2));
    if (!lists.empty())
        std::memcpy(ln.hstage + sd + sj + si, lists.data(), lists.size() * sizeof(int));
    hipStream_t s = ln.s;
    // the windows' events: every append so far (the caller holds amu)
    if (sv->apending) HIPCHK(c, hipStreamWaitEvent(s, sv->aev, 0));
    HIPCHK(c, hipMemcpyAsync(ln.descd.p, ln.hstage, td.size() * sizeof(TileDesc),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(ln.jobsd.p, ln.hstage + sd, bj.size() * sizeof(BJob),
                             hipMemcpyHostToDevice, s));
    if (!items.empty())
        HIPCHK(c, hipMemcpyAsync(ar + o_items, ln.hstage + sd + sj, items.size() * sizeof(int2),
                                 hipMemcpyHostToDevice, s));
    if (!lists.empty())
        HIPCHK(c, hipMemcpyAsync(ar + o_lists, ln.hstage + sd + sj + si,
                                 lists.size() * sizeof(int), hipMemcpyHostToDevice, s));
    BatchDev d;
    d.tiles = (const TileDesc *)ln.descd.p;
    d.jobs = (const BJob *)ln.jobsd.p;
    d.pk = P<int>(sv->pk);
    d.orig = P<int>(sv->origd);
    d.lam = (int *)(ar + o_lam);
    d.tbl = (int2 *)(ar + o_tbl);
    d.status = P<int>(ln.statd);
    d.sparse = c->param[FE_PARAM_TYPE_DISPATCH] != 0;
    d.wpb = WPB;
    int *lists_d = (int *)(ar + o_lists);
    int *fr = (int *)(ar + o_fr), *fx = (int *)(ar + o_fx), *qc = (int *)(ar + o_q);
    const int grid = std::max(1, sv->ncu * sv->cfg.waves_per_cu / WPB);
    launch_fill(qc, 0, NMAX * (1 + NDCLS), s);
    launch_fill(P<int>(ln.statd), 0, 1, s);
    int q = 0;
    for (const LvPlan &L : lp) {
        launch_clear_flags(lists_d + L.pl, (int)L.npl, fr, fx, s);
        launch_plan_batch(d.tiles, d.jobs, P<int>(sv->tileWd), lists_d + L.pl, (int)L.npl, d.lam,
                          s);
        d.items = (const int2 *)(ar + o_items) + L.it_rel;
        d.nitems = (int)L.n_rel;
        d.qctr = qc + q++;
        d.flags = fr;
        launch_persist(L.N, false, 0, d, grid, s);
        launch_concat_batch(d, lists_d + L.pl, (int)L.npl, false, s);
        launch_persist_fixup(L.N, false, 0, d, lists_d + L.pl, (int)L.npl, s);
        d.flags = fx;
        for (int dd = 0; dd < NDCLS; ++dd) {
            if (!L.n_ex[dd]) continue;
            d.items = (const int2 *)(ar + o_items) + L.it_ex[dd];
            d.nitems = (int)L.n_ex[dd];
            d.qctr = qc + q++;
            launch_persist(L.N, true, dd, d, grid, s);
        }
        for (int dd = 0; dd < NDCLS; ++dd)
            if (L.npld[dd]) {
                launch_concat_batch(d, lists_d + L.pld[dd], (int)L.npld[dd], true, s);
                launch_persist_fixup(L.N, true, dd, d, lists_d + L.pld[dd], (int)L.npld[dd], s);
            }
        // deep-class groups: k_deep over each request's window
        for (const GroupDesc &g : sv->groups) {
            if (g.key % NDCLS != DEEP_CLS || g.key / NDCLS + 1 != L.N) continue;
            for (int r = 0; r < R; ++r) {
                // (rings sized at creation for the longest window fit any shorter one)
                const DeepPlan dp = deep_plan(L.N, (int64_t)g.tiles * WAVE, g.dcap, bj[r].n,
                                              (int64_t)ln.deepd.cap);
                if (dp.bytes > (int64_t)ln.deepd.cap)
                    return fail(c, FE_EINTERNAL, "deep rings exceed the lane's scratch");
                DeepArgs a{};
                a.ids = bj[r].ids;
                a.ticks = bj[r].ticks;
                a.n = bj[r].n;
                a.pk = P<int>(sv->pk) + g.rec_base;
                a.orig = P<int>(sv->origd) + (int64_t)g.tile_base * WAVE;
                a.ring = P<int2>(ln.deepd);
                a.out = bj[r].exact;
                a.upper = bj[r].upper;
                a.theta = bj[r].theta;
                a.status = P<int>(ln.statd);
                deep_launch(L.N, a, dp, (int64_t)g.tiles * WAVE, s);
            }
        }
    }
    HIPCHK(c, hipMemcpyAsync(ln.hout, ln.outd.p, (size_t)R * 2 * M * sizeof(int),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(ln.hout + (size_t)R * 2 * M, ln.statd.p, sizeof(int),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(ln.done, s));
    HIPCHK(c, hipGetLastError());
    return FE_OK;
}

void server_loop(fe_server *sv)
{
    fe_ctx *c = sv->c;
    (void)hipSetDevice(c->device);
    const int64_t lane_budget = std::max<int64_t>(1, sv->cfg.hbm_budget / sv->cfg.max_inflight);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool progressed = false;
        // completions
        for (auto &ln : sv->lanes) {
            if (!ln.busy) continue;
            const hipError_t e = hipEventQuery(ln.done);
            if (e == hipErrorNotReady) continue;
            const int64_t now = steady_ns();
            // the round's device status word (a failed device check fails the round)
            const int bits = e == hipSuccess ? ln.hout[ln.reqs.size() * 2 * (size_t)sv->M] : 0;
            for (size_t r = 0; r < ln.reqs.size(); ++r) {
                fe_server::Req *q = ln.reqs[r];
                if (e != hipSuccess) {
                    q->status = FE_EDEVICE;
                } else if (bits) {
                    q->status = status_code(bits);
                } else {
                    const int *u = ln.hout + r * 2 * (size_t)sv->M;
                    q->up.assign(u, u + sv->M);
                    q->ex.assign(u + sv->M, u + 2 * (size_t)sv->M);
                    int ns = 0, nf = 0;
                    for (int m = 0; m < sv->M; ++m) {
                        ns += q->up[m] >= q->r.theta;
                        nf += q->ex[m] >= q->r.theta;
                    }
                    q->ns = ns;
                    q->nf = nf;
                }
                q->done = now;
                q->state = 2;
                sv->st.completed++;
            }
            ln.reqs.clear();
            ln.busy = false;
            progressed = true;
        }
        if (progressed) sv->cv.notify_all();
        // admission into a free lane
        int inflight = 0;
        for (auto &ln : sv->lanes) inflight += ln.busy;
        sv->st.max_inflight_seen = std::max(sv->st.max_inflight_seen, inflight);
        fe_server::Lane *free_lane = nullptr;
        for (auto &ln : sv->lanes)
            if (!ln.busy) {
                free_lane = &ln;
                break;
            }
        if (free_lane && !sv->pending.empty()) {
            int64_t used = 0;
            const int64_t now = steady_ns();
            while (!sv->pending.empty() && (int)free_lane->reqs.size() < sv->cfg.max_round) {
                fe_server::Req *q = sv->pending.front();
                if (!free_lane->reqs.empty() && used + q->foot > lane_budget) {
                    sv->st.budget_closed++;
                    break;
                }
                sv->pending.pop_front();
                used += q->foot;
                q->state = 1;
                q->admit = now;
                free_lane->reqs.push_back(q);
            }
            const int rid = sv->round_id++;
            for (auto *q : free_lane->reqs) {
                q->round = rid;
                q->rsize = (int)free_lane->reqs.size();
            }
            sv->st.rounds++;
            sv->st.largest_round = std::max<int32_t>(sv->st.largest_round,
                                                     (int32_t)free_lane->reqs.size());
            free_lane->busy = true;
            lk.unlock();
            int rc;
            {
                std::lock_guard<std::mutex> ag(sv->amu);
                rc = server_launch(sv, *free_lane);
            }
            lk.lock();
            if (rc != FE_OK) {
                for (auto *q : free_lane->reqs) {
                    q->status = rc;
                    q->state = 2;
                    q->done = steady_ns();
                    sv->st.completed++;
                }
                free_lane->reqs.clear();
                free_lane->busy = false;
                sv->cv.notify_all();
            }
            continue;
        }
        bool any_busy = false;
        for (auto &ln : sv->lanes) any_busy |= ln.busy;
        if (sv->stop && !any_busy && sv->pending.empty()) break;
        if (any_busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            sv->cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

extern "C" int fe_server_create(fe_ctx *c, const fe_server_config *cfg, const int32_t *num_types,
                                const int32_t *types, const int32_t *len, const int32_t *lo,
                                const int32_t *hi, int32_t M, int32_t nmax, fe_server **out)
{
    int rc;
    if (!c || !cfg || !out || !num_types) return FE_EINVAL;
    *out = nullptr;
    if (cfg->n_arrays < 1 || cfg->capacity < 1 || cfg->capacity >= ((int64_t)1 << 31) ||
        cfg->hbm_budget < 1 || cfg->max_inflight < 1 || cfg->max_inflight > 16 ||
        cfg->max_round < 1 || cfg->seg_events < 0 || cfg->waves_per_cu < 0)
        return fail(c, FE_EINVAL, "bad server configuration");
    if (M < 1) return fail(c, FE_EINVAL, "a server needs at least one candidate");
    if ((rc = check_cands(c, types, len, lo, hi, M, nmax))) return rc;
    int maxtypes = 0;
    for (int a = 0; a < cfg->n_arrays; ++a) {
        if (num_types[a] < 1) return fail(c, FE_EINVAL, "num_types must be positive");
        maxtypes = std::max(maxtypes, num_types[a]);
    }
    HIPCHK(c, hipSetDevice(c->device));
    fe_server *sv = new (std::nothrow) fe_server();
    if (!sv) return fail(c, FE_ENOMEM, "host allocation failed");
    sv->c = c;
    sv->cfg = *cfg;
    if (!sv->cfg.seg_events) sv->cfg.seg_events = 16384;
    if (!sv->cfg.waves_per_cu) sv->cfg.waves_per_cu = 16;
    sv->M = M;
    (void)hipDeviceGetAttribute(&sv->ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    auto bail = [&](int code) {
        fe_server_destroy(sv);
        return code;
    };
    // resident candidates: checked on the host, packed once
    const int nm = nmax, hm = std::max(nm - 1, 1);
    std::vector<int> ty((size_t)M * nm), ln(M), lov((size_t)M * hm), hiv((size_t)M * hm);
    HIPCHK(c, hipMemcpy(ty.data(), types, ty.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(ln.data(), len, ln.size() * sizeof(int), hipMemcpyDeviceToHost));
    if (nm > 1) {
        HIPCHK(c, hipMemcpy(lov.data(), lo, (size_t)M * (nm - 1) * sizeof(int), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hiv.data(), hi, (size_t)M * (nm - 1) * sizeof(int), hipMemcpyDeviceToHost));
    }
    std::vector<int> rec, orig, tileW;
    for (int N = 1; N <= nm; ++N) {
        Episodes C;
        C.m = N;
        std::vector<int> back;
        for (int m = 0; m < M; ++m) {
            const int L = ln[m];
            if (L < 1 || L > nm) return bail(fail(c, FE_EINVAL, "bad len"));
            if (L != N) continue;
            int64_t W = 0;
            for (int k = 0; k < N; ++k) {
                const int t = ty[(size_t)m * nm + k];
                if (t < 0 || t >= maxtypes) return bail(fail(c, FE_EINVAL, "type out of range"));
                C.key.push_back(t);
                if (k < N - 1) {
                    const int l = lov[(size_t)m * (nm - 1) + k], h = hiv[(size_t)m * (nm - 1) + k];
                    if (l < 0 || l >= h || h >= TICK_LIMIT)
                        return bail(fail(c, FE_EINVAL, "bad interval"));
                    W += h;
                    C.key.push_back(l);
                    C.key.push_back(h);
                }
            }
            if (W >= TICK_LIMIT) return bail(fail(c, FE_EINVAL, "W too large"));
            back.push_back(m);
        }
        if (back.empty()) continue;
        HostPack hp;
        host_pack(C, nullptr, (int64_t)back.size(), true, hp);
        for (GroupDesc gd : hp.groups) {
            gd.tile_base += sv->ntiles;
            gd.rec_base += (int64_t)rec.size();
            for (int t = 0; t < gd.tiles; ++t) {
                sv->tile_rec.push_back(gd.rec_base + (int64_t)t * rec_ints(N));
                sv->tile_key.push_back(gd.key);
            }
            sv->groups.push_back(gd);
        }
        rec.insert(rec.end(), hp.rec.begin(), hp.rec.end());
        for (int o : hp.orig) orig.push_back(o < 0 ? -1 : back[o]);
        tileW.insert(tileW.end(), hp.tileW.begin(), hp.tileW.end());
        sv->ntiles += hp.tiles;
    }
    if ((rc = ensure(c, sv->pk, rec.size() * sizeof(int)))) return bail(rc);
    if ((rc = ensure(c, sv->origd, orig.size() * sizeof(int)))) return bail(rc);
    if ((rc = ensure(c, sv->tileWd, tileW.size() * sizeof(int)))) return bail(rc);
    HIPCHK(c, hipMemcpy(sv->pk.p, rec.data(), rec.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(sv->origd.p, orig.data(), orig.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(sv->tileWd.p, tileW.data(), tileW.size() * sizeof(int),
                        hipMemcpyHostToDevice));
    // append path
    HIPCHK(c, hipStreamCreateWithFlags(&sv->astream, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&sv->aev, hipEventDisableTiming));
    sv->astage_cap = (size_t)8 << 20;
    if (hipHostMalloc((void **)&sv->astage, sv->astage_cap) != hipSuccess) {
        (void)hipGetLastError();
        sv->astage = nullptr;
        sv->astage_cap = 0;  // synchronous copies only
    }
    // arrays
    sv->arr.resize(cfg->n_arrays);
    for (int a = 0; a < cfg->n_arrays; ++a) {
        sv->arr[a].num_types = num_types[a];
        if ((rc = ensure(c, sv->arr[a].ids, cfg->capacity * sizeof(int)))) return bail(rc);
        if ((rc = ensure(c, sv->arr[a].ticks, cfg->capacity * sizeof(int)))) return bail(rc);
        sv->arr[a].hticks.reserve(std::min<int64_t>(cfg->capacity, 1 << 24));
    }
    // deep-class rings: the largest any round needs (windows of up to capacity events)
    int64_t deep_bytes = 0;
    for (const GroupDesc &g : sv->groups)
        if (g.key % NDCLS == DEEP_CLS)
            deep_bytes = std::max(deep_bytes, deep_plan(g.key / NDCLS + 1, (int64_t)g.tiles * WAVE,
                                                        g.dcap, (int)cfg->capacity).bytes);
    // lanes: stream, completion event, arena sized to the lane's budget
    const int64_t lane_budget = std::max<int64_t>(1, cfg->hbm_budget / cfg->max_inflight);
    const int64_t max_one = req_arena_bytes(sv, (int)cfg->capacity);
    const int64_t arena = std::max<int64_t>(lane_budget, max_one) + (64 << 10);
    sv->lanes.resize(cfg->max_inflight);
    for (auto &L : sv->lanes) {
        HIPCHK(c, hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
        if ((rc = ensure(c, L.arena, arena))) return bail(rc);
        if ((rc = ensure(c, L.outd, (size_t)cfg->max_round * 2 * M * sizeof(int)))) return bail(rc);
        if ((rc = ensure(c, L.descd, (size_t)cfg->max_round * sv->ntiles * sizeof(TileDesc))))
            return bail(rc);
        if ((rc = ensure(c, L.jobsd, (size_t)cfg->max_round * sizeof(BJob)))) return bail(rc);
        if ((rc = ensure(c, L.statd, sizeof(int)))) return bail(rc);
        if (deep_bytes > 0 && (rc = ensure(c, L.deepd, (size_t)deep_bytes))) return bail(rc);
        HIPCHK(c, hipHostMalloc((void **)&L.hout,
                                ((size_t)cfg->max_round * 2 * M + 1) * sizeof(int)));
    }
    sv->th = std::thread(server_loop, sv);
    *out = sv;
    return FE_OK;
}

extern "C" int fe_server_append(fe_server *sv, int32_t a, const int32_t *ids, const int32_t *ticks,
                                int64_t n)
{
    if (!sv) return FE_EINVAL;
    fe_ctx *c = sv->c;
    if (a < 0 || a >= (int)sv->arr.size() || n < 0 || (n > 0 && (!ids || !ticks)))
        return fail(c, FE_EINVAL, "bad append");
    if (n == 0) return FE_OK;
    std::lock_guard<std::mutex> ag(sv->amu);
    fe_server::Arr &A = sv->arr[a];
    if (A.n + n > sv->cfg.capacity) return fail(c, FE_ENOMEM, "array %d buffer full", a);
    int prev = A.n ? A.hticks.back() : 0;
    for (int64_t i = 0; i < n; ++i) {
        if (ids[i] < 0 || ids[i] >= A.num_types || ticks[i] < 0 || ticks[i] >= TICK_LIMIT)
            return fail(c, FE_ERANGE, "event out of range");
        if ((A.n || i) && ticks[i] < prev) return fail(c, FE_EUNSORTED, "events out of order");
        prev = ticks[i];
    }
    HIPCHK(c, hipSetDevice(c->device));
    const size_t bytes = (size_t)n * sizeof(int);
    const size_t need = 2 * ((bytes + 255) & ~(size_t)255);
    if (need <= sv->astage_cap) {
        if (sv->apos + need > sv->astage_cap) {
            // the ring wraps: the copies still reading it must finish first
            HIPCHK(c, hipStreamSynchronize(sv->astream));
            sv->apos = 0;
        }
        char *st = sv->astage + sv->apos;
        std::memcpy(st, ids, bytes);
        std::memcpy(st + need / 2, ticks, bytes);
        HIPCHK(c, hipMemcpyAsync(P<int>(A.ids) + A.n, st, bytes, hipMemcpyHostToDevice,
                                 sv->astream));
        HIPCHK(c, hipMemcpyAsync(P<int>(A.ticks) + A.n, st + need / 2, bytes,
                                 hipMemcpyHostToDevice, sv->astream));
        HIPCHK(c, hipEventRecord(sv->aev, sv->astream));
        sv->apending = true;
        sv->apos += need;
    } else {
        HIPCHK(c, hipMemcpy(P<int>(A.ids) + A.n, ids, bytes, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(P<int>(A.ticks) + A.n, ticks, bytes, hipMemcpyHostToDevice));
    }
    A.hticks.insert(A.hticks.end(), ticks, ticks + n);
    A.n += n;
    return FE_OK;
}

extern "C" int fe_server_submit(fe_server *sv, const fe_request *rq, uint64_t *ticket)
{
    if (!sv || !rq || !ticket) return FE_EINVAL;
    fe_ctx *c = sv->c;
    if (rq->array < 0 || rq->array >= (int)sv->arr.size() || rq->t_end < rq->t_begin)
        return fail(c, FE_EINVAL, "bad request");
    fe_server::Req *q = new (std::nothrow) fe_server::Req();
    if (!q) return fail(c, FE_ENOMEM, "host allocation failed");
    q->r = *rq;
    q->arrival = rq->arrival_ns ? rq->arrival_ns : steady_ns();
    {
        std::lock_guard<std::mutex> ag(sv->amu);
        const std::vector<int> &h = sv->arr[rq->array].hticks;
        q->a = (int)(std::lower_bound(h.begin(), h.end(), rq->t_begin) - h.begin());
        q->b = (int)(std::lower_bound(h.begin(), h.end(), rq->t_end) - h.begin());
    }
    q->foot = req_arena_bytes(sv, q->b - q->a) + 2 * (int64_t)sv->M * 4;
    std::lock_guard<std::mutex> lk(sv->mu);
    q->ticket = sv->next_ticket++;
    sv->reqs[q->ticket] = q;
    sv->st.submitted++;
    if (q->foot > sv->cfg.hbm_budget) {
        q->status = FE_ENOMEM;
        q->state = 2;
        q->done = steady_ns();
        sv->st.rejected++;
        sv->st.completed++;
    } else {
        sv->pending.push_back(q);
    }
    *ticket = q->ticket;
    sv->cv.notify_all();
    return FE_OK;
}

namespace {
void fill_response(const fe_server::Req *q, fe_response *out)
{
    out->status = q->status;
    out->n_events = q->b - q->a;
    out->n_survivors = q->ns;
    out->n_frequent = q->nf;
    out->upper = q->up.empty() ? nullptr : q->up.data();
    out->exact = q->ex.empty() ? nullptr : q->ex.data();
    out->arrival_ns = q->arrival;
    out->admit_ns = q->admit;
    out->done_ns = q->done;
    out->round = q->round;
    out->round_size = q->rsize;
    out->footprint = q->foot;
}
}  // namespace

extern "C" int fe_server_poll(fe_server *sv, uint64_t ticket, fe_response *out)
{
    if (!sv || !out) return FE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return FE_EINVAL;
    if (it->second->state != 2) return FE_EBUSY;
    fill_response(it->second, out);
    return FE_OK;
}

extern "C" int fe_server_wait(fe_server *sv, uint64_t ticket, fe_response *out)
{
    if (!sv || !out) return FE_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return FE_EINVAL;
    fe_server::Req *q = it->second;
    sv->cv.wait(lk, [&] { return q->state == 2; });
    fill_response(q, out);
    return FE_OK;
}

extern "C" int fe_server_release(fe_server *sv, uint64_t ticket)
{
    if (!sv) return FE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end() || it->second->state != 2) return FE_EINVAL;
    delete it->second;
    sv->reqs.erase(it);
    return FE_OK;
}

extern "C" int fe_server_get_stats(fe_server *sv, fe_server_stats *out)
{
    if (!sv || !out) return FE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    return FE_OK;
}

extern "C" int fe_server_destroy(fe_server *sv)
{
    if (!sv) return FE_EINVAL;
    fe_ctx *c = sv->c;
    if (sv->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
            for (auto *q : sv->pending) {
                q->status = FE_EINVAL;
                q->state = 2;
            }
            sv->pending.clear();
        }
        sv->cv.notify_all();
        sv->th.join();
    }
    (void)hipSetDevice(c->device);
    for (auto &L : sv->lanes) {
        if (L.s) (void)hipStreamSynchronize(L.s);
        Buf *bs[] = {&L.arena, &L.outd, &L.descd, &L.jobsd, &L.statd, &L.deepd};
        for (Buf *x : bs)
            if (x->p) (void)hipFree(x->p);
        if (L.hout) (void)hipHostFree(L.hout);
        if (L.hstage) (void)hipHostFree(L.hstage);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.s) (void)hipStreamDestroy(L.s);
    }
    if (sv->astream) (void)hipStreamSynchronize(sv->astream);
    for (auto &A : sv->arr) {
        if (A.ids.p) (void)hipFree(A.ids.p);
        if (A.ticks.p) (void)hipFree(A.ticks.p);
    }
    if (sv->astage) (void)hipHostFree(sv->astage);
    if (sv->aev) (void)hipEventDestroy(sv->aev);
    if (sv->astream) (void)hipStreamDestroy(sv->astream);
    Buf *bs[] = {&sv->pk, &sv->origd, &sv->tileWd};
    for (Buf *x : bs)
        if (x->p) (void)hipFree(x->p);
    for (auto &kv : sv->reqs) delete kv.second;
    delete sv;
    return FE_OK;
}
