// Sanitizer build (ASan + UBSan) of the host-side algorithms of the miner
// (candidate generation, key sorting, run-aligned tiling), checked against
// plain definitions: the join against a double loop over the frequent set,
// the sort against std::sort of the keys, the tiling against its invariants
// (every candidate in exactly one lane, one list-depth class per group,
// records and look-back widths equal to the candidates' keys).
#include "fe_hostalgo.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

using namespace fe;
typedef std::vector<int> IV;

static int fails = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                           \
        }                                                                      \
    } while (0)

static const int ILO[] = {0, 50, 100, 190, 20};
static const int IHI[] = {50, 100, 200, 200, 30};

// sorted, duplicate-free set of m-node keys over T types
static EpisodesT<IV> random_set(std::mt19937 &g, int m, int T, int cnt, int niv)
{
    std::set<std::vector<int>> s;
    for (int i = 0; i < cnt; ++i) {
        std::vector<int> k;
        for (int j = 0; j < m; ++j) {
            k.push_back((int)(g() % T));
            if (j + 1 < m) {
                const int v = (int)(g() % niv);
                k.push_back(ILO[v]);
                k.push_back(IHI[v]);
            }
        }
        s.insert(k);
    }
    EpisodesT<IV> E;
    E.m = m;
    for (auto &k : s) E.key.insert(E.key.end(), k.begin(), k.end());
    return E;
}

static void check_join(std::mt19937 &g)
{
    for (int trial = 0; trial < 60; ++trial) {
        const int m = 2 + trial % 4, T = 2 + trial % 3;
        EpisodesT<IV> F = random_set(g, m, T, 20 + trial * 7, 2 + trial % 3);
        EpisodesT<IV> C;
        gen_join(F, C);
        // the definition: alpha + beta's last node, for every beta whose first
        // m-1 nodes and hops equal alpha's last m-1, alpha-major, in F's order
        const int w = 3 * m - 2, ov = 3 * m - 5;
        IV want;
        for (size_t a = 0; a < F.count(); ++a)
            for (size_t b = 0; b < F.count(); ++b) {
                const int *al = F.at(a), *be = F.at(b);
                bool eq = true;
                for (int k = 0; k < ov; ++k) eq &= al[3 + k] == be[k];
                if (!eq) continue;
                want.push_back(al[0]);
                want.push_back(al[1]);
                want.push_back(al[2]);
                want.insert(want.end(), be, be + w);
            }
        CHECK(C.m == m + 1);
        CHECK(C.key == want);
        std::vector<int64_t> first, off;
        CHECK(gen_join_plan(F, first, off) == (int64_t)C.count());
    }
    std::vector<int> F1 = {0, 3, 5};
    std::vector<int> lo = {0, 50}, hi = {50, 100};
    EpisodesT<IV> C2;
    gen_level2(F1, lo, hi, C2);
    CHECK(C2.count() == 3 * 3 * 2);
    CHECK(C2.at(0)[0] == 0 && C2.at(0)[3] == 0 && C2.at(17)[0] == 5 && C2.at(17)[2] == 100);
}

static void check_sort(std::mt19937 &g)
{
    for (int trial = 0; trial < 30; ++trial) {
        const int m = 1 + trial % 5;
        EpisodesT<IV> E = random_set(g, m, 4, 50, 3);
        // shuffle, attach values, sort back
        const size_t F = E.count(), w = 3 * m - 2;
        std::vector<size_t> p(F);
        for (size_t i = 0; i < F; ++i) p[i] = i;
        std::shuffle(p.begin(), p.end(), g);
        EpisodesT<IV> S;
        S.m = m;
        std::vector<int> va, vb;
        for (size_t i : p) {
            S.key.insert(S.key.end(), E.at(i), E.at(i) + w);
            va.push_back((int)i);
            vb.push_back((int)(7 * i + 1));
        }
        sort_episodes(S, &va, &vb);
        CHECK(S.key == E.key);
        for (size_t i = 0; i < F; ++i) CHECK(va[i] == (int)i && vb[i] == (int)(7 * i + 1));
    }
}

static void check_order_by_index(std::mt19937 &g)
{
    for (int trial = 0; trial < 30; ++trial) {
        const int m = 1 + trial % 5;
        EpisodesT<IV> E = random_set(g, m, 4, 50, 3);  // sorted, distinct
        const size_t F = E.count(), w = 3 * m - 2;
        // E's entries are candidates 3i + (i % 2) of a larger, key-ordered
        // set; they arrive in shuffled order with their indices
        std::vector<size_t> p(F);
        for (size_t i = 0; i < F; ++i) p[i] = i;
        std::shuffle(p.begin(), p.end(), g);
        EpisodesT<IV> S;
        S.m = m;
        std::vector<int> sel, va;
        for (size_t i : p) {
            S.key.insert(S.key.end(), E.at(i), E.at(i) + w);
            sel.push_back((int)(3 * i + i % 2));
            va.push_back((int)i);
        }
        order_by_index(S, sel, (int64_t)(3 * F + 2), &va, nullptr);
        CHECK(S.key == E.key);
        for (size_t i = 0; i < F; ++i) CHECK(va[i] == (int)i);
    }
}

static void check_pack(std::mt19937 &g)
{
    for (int trial = 0; trial < 40; ++trial) {
        const int m = 2 + trial % 4;
        // sibling runs: shared first m-1 types, run lengths up to 300
        EpisodesT<IV> C;
        C.m = m;
        int n = 0;
        while (n < 2000 + trial * 50) {
            const int len = 1 + (int)(g() % 300);
            std::vector<int> pre;
            for (int j = 0; j < m - 1; ++j) pre.push_back((int)(g() % 6));
            for (int r = 0; r < len; ++r, ++n) {
                for (int j = 0; j < m; ++j) {
                    C.key.push_back(j < m - 1 ? pre[j] : (int)(g() % 6));
                    if (j + 1 < m) {
                        const int v = (int)(g() % 5);
                        C.key.push_back(ILO[v]);
                        C.key.push_back(IHI[v]);
                    }
                }
            }
        }
        const bool exact = trial % 2 == 0;
        IV order;
        const bool sub = trial % 3 == 0;
        if (sub)
            for (int i = 0; i < n; ++i)
                if (g() % 3) order.push_back(i);
        const int64_t cnt = sub ? (int64_t)order.size() : n;
        HostPackT<IV> hp;
        const int wb = trial % 4 == 1 ? 1000 : -1;
        host_pack(C, sub ? order.data() : nullptr, cnt, exact, hp, wb);
        CHECK((int64_t)hp.orig.size() == (int64_t)hp.tiles * WAVE);
        std::vector<int> seen(n, 0);
        for (int o : hp.orig)
            if (o >= 0) {
                CHECK(o < n);
                if (o < n) seen[o]++;
            }
        for (int i = 0; i < n; ++i) {
            const bool in = !sub || std::binary_search(order.begin(), order.end(), i);
            CHECK(seen[i] == (in ? 1 : 0));
        }
        int tiles = 0;
        for (const GroupDesc &gd : hp.groups) {
            CHECK(gd.tile_base == tiles);
            tiles += gd.tiles;
            const int cls = gd.key % NDCLS;
            CHECK(gd.key / NDCLS + 1 == m);
            for (int t = gd.tile_base; t < gd.tile_base + gd.tiles; ++t)
                for (int l = 0; l < WAVE; ++l) {
                    const int o = hp.orig[(size_t)t * WAVE + l];
                    if (o < 0) continue;
                    CHECK(host_dcls(C.at(o), m, exact) == cls);
                    if (wb >= 0) continue;
                    const int *rec = hp.rec.data() + gd.rec_base + (int64_t)(t - gd.tile_base) *
                                                                       rec_ints(m);
                    for (int k = 0; k < m; ++k) CHECK(rec[k * WAVE + l] == C.at(o)[3 * k]);
                    for (int k = 0; k < m - 1; ++k) {
                        CHECK(rec[(m + k) * WAVE + l] == C.at(o)[3 * k + 1]);
                        CHECK(rec[(2 * m - 1 + k) * WAVE + l] == C.at(o)[3 * k + 2]);
                    }
                }
        }
        CHECK(tiles == hp.tiles);
    }
}

int main()
{
    std::mt19937 g(12345);
    check_join(g);
    check_sort(g);
    check_order_by_index(g);
    check_pack(g);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host algorithms: all checks passed\n");
    return 0;
}
