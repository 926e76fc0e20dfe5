// fe_hostalgo.h -- host-side algorithms of the level-wise miner and of the
// batch / server planning: candidate generation (Problem 1's level-wise
// scheme, Sec. 5 intro), sorting of episode keys, and run-aligned tiling of
// candidates for the Map kernels.  Plain C++ (standard library only), so the
// sanitizer build of the test suite compiles it without HIP.  IV is the int
// vector type (the library uses one with a pinned, non-initialising
// allocator for large arrays).
#pragma once

#include "fe_const.h"

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace fe {

// One candidate group (episode size and list-depth class) already packed
// in the tile table: tiles [tile_base, tile_base+tiles), records from int
// offset rec_base, widest W (sum of hi) wmax, real candidates ncand, and
// for the deep class the largest window bound of its hops (dcap).
struct GroupDesc {
    int key;
    int tiles;
    int tile_base;
    int64_t rec_base;
    int wmax;
    int64_t ncand;
    int dcap = 0;
};

// Host worker threads for candidate generation and packing.
inline int host_threads()
{
    static const int n = [] {
        const unsigned h = std::thread::hardware_concurrency();
        return (int)std::max(1u, std::min(16u, h ? h : 1u));
    }();
    return n;
}

// f(begin, end, part) over [0, n) split into contiguous parts, in parallel
// when each part gets at least `grain` items.
template <class F> int par_for(int64_t n, int64_t grain, F &&f)
{
    const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / grain));
    if (parts <= 1) {
        f((int64_t)0, n, 0);
        return 1;
    }
    std::vector<std::thread> th;
    th.reserve(parts);
    for (int q = 0; q < parts; ++q)
        th.emplace_back([&f, n, parts, q] { f(n * q / parts, n * (q + 1) / parts, q); });
    for (auto &t : th) t.join();
    return parts;
}

// Order-preserving parallel filter of [0, n): the indices i with keep(i).
template <class P, class IV> void par_select(int64_t n, P &&keep, IV &out)
{
    const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / 65536));
    std::vector<int64_t> cnt(parts + 1, 0);
    par_for(n, (n + parts - 1) / std::max(parts, 1), [&](int64_t b, int64_t e, int q) {
        int64_t k = 0;
        for (int64_t i = b; i < e; ++i) k += keep(i) ? 1 : 0;
        cnt[q + 1] = k;
    });
    for (int q = 0; q < parts; ++q) cnt[q + 1] += cnt[q];
    out.resize(cnt[parts]);
    par_for(n, (n + parts - 1) / std::max(parts, 1), [&](int64_t b, int64_t e, int q) {
        int64_t k = cnt[q];
        for (int64_t i = b; i < e; ++i)
            if (keep(i)) out[k++] = (int)i;
    });
}

// An episode of size m is keyed by its interleaved tuple
// (E1, lo1, hi1, E2, ..., lo_(m-1), hi_(m-1), E_m): 3m-2 ints.  The prefix
// (first m-1 nodes) is the first 3m-5 ints, the suffix (last m-1 nodes)
// the last 3m-5 ints.
template <class IV> struct EpisodesT {
    int m = 0;  // episode size
    IV key;     // [count * (3m-2)]
    size_t count() const { return m ? key.size() / (3 * m - 2) : 0; }
    const int *at(size_t i) const { return key.data() + i * (3 * m - 2); }
};

template <class IV> void sort_episodes(EpisodesT<IV> &E, std::vector<int> *vals_a, std::vector<int> *vals_b)
{
    const int w = 3 * E.m - 2;
    const size_t F = E.count();
    std::vector<size_t> idx(F);
    for (size_t i = 0; i < F; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        return std::lexicographical_compare(E.at(a), E.at(a) + w, E.at(b), E.at(b) + w);
    });
    IV k2(E.key.size());
    std::vector<int> a2(vals_a ? F : 0), b2(vals_b ? F : 0);
    for (size_t i = 0; i < F; ++i) {
        std::memcpy(k2.data() + i * w, E.at(idx[i]), w * sizeof(int));
        if (vals_a) a2[i] = (*vals_a)[idx[i]];
        if (vals_b) b2[i] = (*vals_b)[idx[i]];
    }
    E.key.swap(k2);
    if (vals_a) vals_a->swap(a2);
    if (vals_b) vals_b->swap(b2);
}

// Reorder E's entries, given in the order of their candidate indices sel
// (distinct, below M), into increasing index order, and the values with
// them: when the candidates were generated in key order this sorts E in
// O(M/64 + F) -- the rank of an index is found in a bitmap of the selected
// indices with per-word prefix counts.
template <class IV>
void order_by_index(EpisodesT<IV> &E, const std::vector<int> &sel, int64_t M,
                    std::vector<int> *vals_a, std::vector<int> *vals_b)
{
    const int w = 3 * E.m - 2;
    const size_t F = E.count();
    std::vector<uint64_t> bm((size_t)((M + 63) / 64), 0);
    for (size_t k = 0; k < F; ++k) bm[(size_t)sel[k] >> 6] |= 1ull << (sel[k] & 63);
    std::vector<int64_t> pre(bm.size() + 1, 0);
    for (size_t j = 0; j < bm.size(); ++j) pre[j + 1] = pre[j] + __builtin_popcountll(bm[j]);
    IV k2(E.key.size());
    std::vector<int> a2(vals_a ? F : 0), b2(vals_b ? F : 0);
    // (distinct destinations: the scatter runs on every host thread)
    par_for((int64_t)F, 65536, [&](int64_t b, int64_t e, int) {
        for (int64_t k = b; k < e; ++k) {
            const int x = sel[k];
            const size_t d = (size_t)(pre[(size_t)x >> 6] +
                                      __builtin_popcountll(bm[(size_t)x >> 6] &
                                                           ((1ull << (x & 63)) - 1ull)));
            std::memcpy(k2.data() + d * w, E.at(k), w * sizeof(int));
            if (vals_a) a2[d] = (*vals_a)[k];
            if (vals_b) b2[d] = (*vals_b)[k];
        }
    });
    E.key.swap(k2);
    if (vals_a) vals_a->swap(a2);
    if (vals_b) vals_b->swap(b2);
}

// Level 2: every ordered pair of frequent types (repeats allowed) times
// every interval of I.
template <class IV>
void gen_level2(const std::vector<int> &F1, const std::vector<int> &ilo,
                const std::vector<int> &ihi, EpisodesT<IV> &out)
{
    out.m = 2;
    out.key.clear();
    out.key.reserve(F1.size() * F1.size() * ilo.size() * 4);
    for (int a : F1)
        for (int b : F1)
            for (size_t k = 0; k < ilo.size(); ++k) {
                out.key.push_back(a);
                out.key.push_back(ilo[k]);
                out.key.push_back(ihi[k]);
                out.key.push_back(b);
            }
}

// Level m+1 from the sorted frequent set of size m: alpha joined with every
// beta whose first m-1 nodes and intervals equal alpha's last m-1, in the
// order (alpha, beta).  Each alpha's betas are one contiguous range of F;
// ranges are found and written in parallel.
// Range search of the join: for each alpha of F (sorted), first[a] = the
// first beta whose first m-1 nodes and hops equal alpha's last m-1, and
// alpha's candidates are outputs off[a]..off[a+1]; returns off[cnt].
template <class IV>
int64_t gen_join_plan(const EpisodesT<IV> &F, std::vector<int64_t> &first, std::vector<int64_t> &off)
{
    const int m = F.m, ov = 3 * m - 5;
    const int64_t cnt = (int64_t)F.count();
    first.assign(cnt, 0);
    off.assign(cnt + 1, 0);
    // F is sorted, so equal prefixes (first m-1 nodes and hops) are runs:
    // their starts, and the distinct prefixes packed for the searches
    IV starts;
    par_select(cnt, [&](int64_t i) {
        return i == 0 || !std::equal(F.at(i - 1), F.at(i - 1) + ov, F.at(i));
    }, starts);
    const int64_t U = (int64_t)starts.size();
    std::vector<int> up((size_t)U * ov);
    for (int64_t q = 0; q < U; ++q) std::memcpy(up.data() + q * ov, F.at(starts[q]), ov * sizeof(int));
    par_for(cnt, 4096, [&](int64_t b, int64_t e, int) {
        for (int64_t a = b; a < e; ++a) {
            const int *suf = F.at(a) + 3;
            int64_t lo = 0, hi = U;  // first distinct prefix >= suf
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int *pm = up.data() + mid * ov;
                if (std::lexicographical_compare(pm, pm + ov, suf, suf + ov))
                    lo = mid + 1;
                else
                    hi = mid;
            }
            const bool hit = lo < U && std::equal(suf, suf + ov, up.data() + lo * ov);
            first[a] = lo < U ? starts[lo] : cnt;
            off[a + 1] = hit ? (lo + 1 < U ? starts[lo + 1] : cnt) - starts[lo] : 0;
        }
    });
    for (int64_t a = 0; a < cnt; ++a) off[a + 1] += off[a];
    return off[cnt];
}

template <class IV> void gen_join(const EpisodesT<IV> &F, EpisodesT<IV> &out)
{
    const int m = F.m, w = 3 * m - 2, wo = w + 3;
    out.m = m + 1;
    const int64_t cnt = (int64_t)F.count();
    std::vector<int64_t> first, off;
    gen_join_plan(F, first, off);
    out.key.resize((size_t)off[cnt] * wo);
    par_for(cnt, 4096, [&](int64_t b, int64_t e, int) {
        for (int64_t a = b; a < e; ++a) {
            int *o = out.key.data() + (size_t)off[a] * wo;
            const int *al = F.at(a);
            for (int64_t j = 0; j < off[a + 1] - off[a]; ++j, o += wo) {
                o[0] = al[0];
                o[1] = al[1];
                o[2] = al[2];
                std::memcpy(o + 3, F.at(first[a] + j), w * sizeof(int));
            }
        }
    });
}

// Host-side tiling of a level's candidates (all of size m) for the Map
// kernels, in the packed tile layout the device grouping produces:
// candidates are grouped by list-depth class; inside a group, maximal runs
// of join siblings (same first m-1 types, consecutive in generation order)
// fill whole tiles, so those waves take the shared-prefix path; a run's
// remainder of at least half a tile gets a padded tile of its own, shorter
// remainders are packed together after every run's tiles.
template <class IV> struct HostPackT {
    IV rec, orig, tileW;
    std::vector<GroupDesc> groups;
    int tiles = 0;
};

// largest window bound of an episode key's hops
inline int host_bound(const int *k, int m)
{
    int bound = 1;
    for (int j = 0; j < m - 1; ++j) bound = std::max(bound, window_bound(k[3 * j + 1], k[3 * j + 2]));
    return bound;
}

inline int host_dcls(const int *k, int m, bool exact)
{
    return exact ? depth_class(host_bound(k, m)) : 0;
}

// order: the candidates to pack (indices into C), or null for all of C in
// order; n: their number.  With wmax_bound >= 0 only the lane assignment
// (hp.orig) and the groups are produced, each group's wmax set to that bound;
// the records are then built on the device (k_build_rec) from C's keys.
template <class IV>
void host_pack(const EpisodesT<IV> &C, const int *order, int64_t n, bool exact, HostPackT<IV> &hp,
               int wmax_bound = -1, IV *lane_pool = nullptr)
{
    const int m = C.m;
    const int ri = rec_ints(m);
    hp.rec.clear();
    hp.orig.clear();
    hp.tileW.clear();
    hp.groups.clear();
    hp.tiles = 0;
    auto cand = [&](int64_t i) { return order ? order[i] : (int)i; };
    // depth classes, stable (all of C in order: one class, the identity)
    const bool ident = !exact && !order;
    IV byc[NDCLS];
    if (!exact && !ident) {
        byc[0].resize(n);
        par_for(n, 65536, [&](int64_t b, int64_t e, int) {
            for (int64_t i = b; i < e; ++i) byc[0][i] = cand(i);
        });
    } else if (exact) {
        // one pass counting per part and class, then a stable scatter
        IV cls(n);
        const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(),
                                                                        n / 65536));
        std::vector<int64_t> cnt((size_t)parts * NDCLS, 0);
        auto range = [&](int q, int64_t &b, int64_t &e) {
            b = n * q / parts;
            e = n * (q + 1) / parts;
        };
        par_for(parts, 1, [&](int64_t q0, int64_t q1, int) {
            for (int64_t q = q0; q < q1; ++q) {
                int64_t b, e;
                range((int)q, b, e);
                for (int64_t i = b; i < e; ++i) {
                    cls[i] = host_dcls(C.at(cand(i)), m, true);
                    ++cnt[q * NDCLS + cls[i]];
                }
            }
        });
        std::vector<int64_t> off((size_t)parts * NDCLS);
        for (int k = 0; k < NDCLS; ++k) {
            int64_t acc = 0;
            for (int q = 0; q < parts; ++q) {
                off[q * NDCLS + k] = acc;
                acc += cnt[q * NDCLS + k];
            }
            byc[k].resize(acc);
        }
        par_for(parts, 1, [&](int64_t q0, int64_t q1, int) {
            for (int64_t q = q0; q < q1; ++q) {
                int64_t b, e;
                range((int)q, b, e);
                int64_t o[NDCLS];
                for (int k = 0; k < NDCLS; ++k) o[k] = off[q * NDCLS + k];
                for (int64_t i = b; i < e; ++i) byc[cls[i]][o[cls[i]]++] = cand(i);
            }
        });
    }
    auto same_prefix = [&](int a, int b) {
        const int *x = C.at(a), *y = C.at(b);
        for (int j = 0; j < m - 1; ++j)
            if (x[3 * j] != y[3 * j]) return false;
        return true;
    };
    for (int cls = 0; cls < NDCLS; ++cls) {
        const IV &v = byc[cls];
        const int64_t V = ident ? (cls == 0 ? n : 0) : (int64_t)v.size();
        if (V == 0) continue;
        auto vat = [&](int64_t i) { return ident ? (int)i : v[i]; };
        // copy v[s0, s0+len) to dst
        auto vcopy = [&](int *dst, int64_t s0, int64_t len) {
            if (ident)
                for (int64_t j = 0; j < len; ++j) dst[j] = (int)(s0 + j);
            else
                std::memcpy(dst, v.data() + s0, len * sizeof(int));
        };
        // runs of equal first m-1 types
        IV starts;
        par_select(V, [&](int64_t i) { return i == 0 || !same_prefix(vat(i - 1), vat(i)); },
                   starts);
        const int64_t R = (int64_t)starts.size();
        std::vector<int64_t> toff(R + 1, 0), moff(R + 1, 0);
        for (int64_t r = 0; r < R; ++r) {
            const int64_t len = (r + 1 < R ? starts[r + 1] : V) - starts[r];
            const int64_t rem = len % WAVE;
            toff[r + 1] = toff[r] + len / WAVE + (rem >= WAVE / 2 ? 1 : 0);
            moff[r + 1] = moff[r] + (rem >= WAVE / 2 ? 0 : rem);
        }
        const int64_t run_tiles = toff[R], nmixed = moff[R];
        const int tiles = (int)(run_tiles + (nmixed + WAVE - 1) / WAVE);
        IV lanes;
        if (lane_pool && hp.orig.empty()) lanes.swap(*lane_pool);
        lanes.resize((size_t)tiles * WAVE);
        par_for(R, 1024, [&](int64_t b, int64_t e, int) {
            for (int64_t r = b; r < e; ++r) {
                const int64_t s0 = starts[r], len = (r + 1 < R ? starts[r + 1] : V) - s0;
                const int64_t full = len / WAVE * WAVE, rem = len - full;
                int *dst = lanes.data() + toff[r] * WAVE;
                vcopy(dst, s0, full);
                if (rem >= WAVE / 2) {
                    vcopy(dst + full, s0 + full, rem);
                    std::fill(dst + full + rem, dst + full + WAVE, -1);
                } else {
                    vcopy(lanes.data() + run_tiles * WAVE + moff[r], s0 + full, rem);
                }
            }
        });
        std::fill(lanes.begin() + run_tiles * WAVE + nmixed, lanes.end(), -1);
        int dcap = 0;  // largest window bound of the deep class
        if (exact && cls == DEEP_CLS)
            for (int64_t i = 0; i < V; ++i) dcap = std::max(dcap, host_bound(C.at(vat(i)), m));
        if (wmax_bound >= 0) {
            GroupDesc gd{(m - 1) * NDCLS + cls, tiles, hp.tiles, (int64_t)hp.tiles * ri,
                         wmax_bound, V, dcap};
            if (hp.orig.empty()) hp.orig.swap(lanes);
            else hp.orig.insert(hp.orig.end(), lanes.begin(), lanes.end());
            hp.tiles += tiles;
            hp.groups.push_back(gd);
            continue;
        }
        GroupDesc gd{(m - 1) * NDCLS + cls, tiles, hp.tiles, (int64_t)hp.rec.size(), 0, V, dcap};
        const size_t rec0 = hp.rec.size(), orig0 = hp.orig.size(), tw0 = hp.tileW.size();
        hp.rec.resize(rec0 + (size_t)tiles * ri);
        hp.orig.resize(orig0 + (size_t)tiles * WAVE);
        hp.tileW.resize(tw0 + tiles);
        par_for(tiles, 256, [&](int64_t t0, int64_t t1, int) {
            for (int64_t t = t0; t < t1; ++t) {
                int *rec = hp.rec.data() + rec0 + (size_t)t * ri;
                int W = 0;
                for (int l = 0; l < WAVE; ++l) {
                    const int idx = lanes[(size_t)t * WAVE + l];
                    hp.orig[orig0 + (size_t)t * WAVE + l] = idx;
                    if (idx < 0) {
                        for (int k = 0; k < m; ++k) rec[k * WAVE + l] = -1;
                        for (int k = 0; k < m - 1; ++k) {
                            rec[(m + k) * WAVE + l] = 0;
                            rec[(2 * m - 1 + k) * WAVE + l] = 0;
                        }
                        continue;
                    }
                    const int *key = C.at(idx);
                    int w = 0;
                    for (int k = 0; k < m; ++k) rec[k * WAVE + l] = key[3 * k];
                    for (int k = 0; k < m - 1; ++k) {
                        rec[(m + k) * WAVE + l] = key[3 * k + 1];
                        rec[(2 * m - 1 + k) * WAVE + l] = key[3 * k + 2];
                        w += key[3 * k + 2];
                    }
                    W = std::max(W, w);
                }
                hp.tileW[tw0 + t] = W;
            }
        });
        for (int t = 0; t < tiles; ++t) gd.wmax = std::max(gd.wmax, hp.tileW[tw0 + t]);
        hp.tiles += tiles;
        hp.groups.push_back(gd);
    }
}


}  // namespace fe
