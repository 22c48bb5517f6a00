// Host-only checks of the library's planning code and leaf arithmetic, built
// with g++ under the address and undefined-behaviour sanitizers (no GPU, no
// HIP headers).  Modes:
//   plan    random batches: tree tables and block-to-merge maps are complete,
//           consistent and in bounds; every level's merges have finished
//           children; workspace, checkpoint and reverse-pass carvings are
//           aligned, disjoint and inside the sizes they report.
//   leaf    reads "n d_0..d_(n-1) e_0..e_(n-2)" from stdin, runs the leaf
//           QL (rows 0 and n-1 tracked) and prints status, eigenvalues and
//           the two rows.
//   search  the assembly's partition-point searches (binary and 8-way, over
//           plain lists and over roots given as origin + tau) against a
//           linear count, on ascending lists with repeated values.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <vector>

#define TDE_DEV inline
#define TDE_RCP_ESTIMATE(x) (1.0 / (x))
// a single-precision estimate, as coarse as the hardware one, so the Newton steps are exercised
#define TDE_RSQ_ESTIMATE(x) ((1.0 / std::sqrt(x)) * (1.0 + 3e-8))
#include "../../paper_2605_26599_amd/csrc/tde_device.h"
#include "../../paper_2605_26599_amd/csrc/tde_plan.h"
#include "../../paper_2605_26599_amd/csrc/tde_tree.h"

using namespace tde;

static int g_fail = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                         \
            return;                                                           \
        }                                                                     \
    } while (0)

static void check_plan(const std::vector<long long>& offs, int leaf, bool dc) {
    Plan p;
    p.leaf = leaf;
    p.leaf_dc = dc;
    p.offs = offs;
    CHECK(plan_host(&p) == 0);
    const long long n = offs.back();
    CHECK(p.ntot == n);
    // leaves partition the columns of every problem
    std::vector<int> cover((size_t)(n > 0 ? n : 1), 0);
    for (const LeafRec& L : p.h_leaves) {
        CHECK(L.size >= 1 && L.size <= leaf);
        CHECK(L.off >= offs[L.prob] && L.off + L.size <= offs[L.prob + 1]);
        for (int i = 0; i < L.size; ++i) cover[(size_t)(L.off + i)]++;
    }
    for (long long i = 0; i < n; ++i) CHECK(cover[(size_t)i] == 1);
    // merges: children complete before the parent's level, packing consistent
    std::set<std::pair<long long, long long>> done;  // finished nodes (off, size)
    for (const LeafRec& L : p.h_leaves) done.insert({L.off, (long long)L.size});
    size_t bi = 0;
    for (size_t h = 0; h < p.levels.size(); ++h) {
        const LevelInfo& I = p.levels[h];
        CHECK(I.mstart >= 0 && I.mstart + I.M <= (int)p.h_merges.size());
        long long pk = 0;
        int smax = 0;
        bool all_root = true;
        std::vector<std::pair<long long, long long>> made;
        for (int m = 0; m < I.M; ++m) {
            const MergeRec& R = p.h_merges[(size_t)(I.mstart + m)];
            CHECK(R.nL >= 1 && R.nR >= 1 && R.nR - R.nL >= 0 && R.nR - R.nL <= 1);
            CHECK(R.pk == pk);
            CHECK(done.count({R.off, (long long)R.nL}) && done.count({R.off + R.nL, (long long)R.nR}));
            CHECK(R.off >= offs[R.prob] && R.off + R.nL + R.nR <= offs[R.prob + 1]);
            const bool whole = (R.off == offs[R.prob] && R.off + R.nL + R.nR == offs[R.prob + 1]);
            CHECK(((R.flags & MF_ROOT) != 0) == whole);
            all_root = all_root && whole;
            pk += R.nL + R.nR;
            smax = std::max(smax, R.nL + R.nR);
            made.push_back({R.off, (long long)(R.nL + R.nR)});
        }
        CHECK(pk == I.N && smax == I.smax);
        CHECK((I.all_root != 0) == all_root);  // levels whose Loewner and row steps are skipped
        for (auto& x : made) done.insert(x);
        // block-to-merge map: entry b names the merge holding column min(b*kWG, N-1)
        CHECK(I.bstart == (int)bi);
        const long long nb = (I.N + kWG - 1) / kWG;
        for (long long b = 0; b <= nb; ++b) {
            CHECK(bi < p.h_blkm.size());
            const int m = p.h_blkm[bi++];
            CHECK(m >= 0 && m < I.M);
            const long long c = std::min(b * (long long)kWG, I.N - 1);
            const MergeRec& R = p.h_merges[(size_t)(I.mstart + m)];
            CHECK(R.pk <= c && c < R.pk + R.nL + R.nR);
        }
        // in-wave packs (levels of merges of at most kLeafMax columns): ascending
        // first merges from 0, then M; each pack at most kLeafMax columns, and no
        // pack could have taken its successor's first merge
        CHECK(I.wpstart == (int)bi);
        if (I.smax <= kLeafMax) {
            CHECK(I.nwp >= 1 && bi + (size_t)I.nwp + 1 <= p.h_blkm.size());
            CHECK(p.h_blkm[bi] == 0 && p.h_blkm[bi + (size_t)I.nwp] == I.M);
            for (int k = 0; k < I.nwp; ++k) {
                const int a = p.h_blkm[bi + (size_t)k], z = p.h_blkm[bi + (size_t)k + 1];
                CHECK(a < z);
                const MergeRec& A = p.h_merges[(size_t)(I.mstart + a)];
                const MergeRec& Z = p.h_merges[(size_t)(I.mstart + z - 1)];
                const long long cols = Z.pk + Z.nL + Z.nR - A.pk;
                CHECK(cols <= kLeafMax);
                if (z < I.M) {
                    const MergeRec& F = p.h_merges[(size_t)(I.mstart + z)];
                    CHECK(cols + F.nL + F.nR > kLeafMax);
                }
            }
            bi += (size_t)I.nwp + 1;
        } else {
            CHECK(I.nwp == 0);
        }
    }
    CHECK(bi == p.h_blkm.size());
    // every problem of more than `leaf` columns ends with its root merge
    for (size_t b = 0; b + 1 < offs.size(); ++b)
        if (offs[b + 1] - offs[b] > leaf) CHECK(done.count({offs[b], offs[b + 1] - offs[b]}));
    if (dc) {
        CHECK((int)p.h_shdr.size() == kLeafMax + 1);
        for (int l = 1; l <= kLeafMax; ++l) {
            const SubHdr& H = p.h_shdr[(size_t)l];
            CHECK(H.H >= 0 && H.H < 8);
            CHECK(H.mbase + H.lv[H.H] <= (int)p.h_smer.size());
            for (int k = 0; k < H.H; ++k) CHECK(H.lv[k] <= H.lv[k + 1]);
            for (int q = 0; q < H.lv[H.H]; ++q) {
                const SubMerge& S = p.h_smer[(size_t)(H.mbase + q)];
                CHECK(S.off + S.nL + S.nR <= l);
            }
        }
    }
    // carvings: aligned, disjoint and inside the reported size
    const long long B = (long long)offs.size() - 1;
    struct Slice {
        size_t a, b;
    };
    const size_t wsz = workspace_layout(n, B, n, nullptr, nullptr);
    std::vector<char> buf(wsz + 256);
    char* base = (char*)(((uintptr_t)buf.data() + 255) & ~(uintptr_t)255);
    Work w{};
    CHECK(workspace_layout(n, B, n, base, &w) == wsz);
    CHECK(w.sec_cap == kSecMaxIter);
    const long long nn = n > 0 ? n : 1;
    std::vector<Slice> sl;
    auto add = [&](const void* p0, size_t bytes) { sl.push_back({(size_t)((const char*)p0 - base), bytes}); };
    add(w.lam, 8 * nn); add(w.blo, 8 * nn); add(w.bhi, 8 * nn); add(w.D, 8 * nn); add(w.Z, 8 * nn);
    add(w.RL, 8 * nn); add(w.RH, 8 * nn); add(w.src, 4 * nn); add(w.D2, 8 * nn); add(w.Z2, 8 * nn);
    add(w.RL2, 8 * nn); add(w.RH2, 8 * nn); add(w.st, 4 * nn); add(w.scan, 4 * (nn + nn / 2 + 2));
    add(w.scanC, 4 * (nn + nn / 2 + 2)); add(w.scanR, 4 * (nn + nn / 2 + 2)); add(w.nnpos, 4 * nn);
    add(w.cf, 4 * nn); add(w.Da, 8 * nn); add(w.Za, 8 * nn); add(w.Wa, 8 * nn); add(w.RLa, 8 * nn);
    add(w.RHa, 8 * nn); add(w.amerge, 4 * nn); add(w.apos, 4 * nn); add(w.rpos, 4 * nn);
    add(w.dpos, 4 * nn); add(w.org, 4 * nn); add(w.tau, 8 * nn); add(w.rootval, 8 * nn);
    add(w.dorg, 8 * nn); add(w.zhat, 8 * nn); add(w.PBL, 8 * nn); add(w.PBH, 8 * nn); add(w.Dd, 8 * nn);
    add(w.RLd, 8 * nn); add(w.RHd, 8 * nn); add(w.Dr, 8 * nn); add(w.RLr, 8 * nn); add(w.RHr, 8 * nn);
    add(w.pmax, 8 * (size_t)(B > 0 ? B : 1));
    std::sort(sl.begin(), sl.end(), [](const Slice& x, const Slice& y) { return x.a < y.a; });
    for (size_t k = 0; k < sl.size(); ++k) {
        CHECK(sl[k].a % 256 == 0);
        CHECK(sl[k].a + sl[k].b <= wsz);
        if (k + 1 < sl.size()) CHECK(sl[k].a + sl[k].b <= sl[k + 1].a);
    }
    std::memset(base, 0, wsz);  // every byte of the reported size is addressable
    const size_t gsz = grad_layout(n, p.nmerges, nullptr, nullptr);
    std::vector<char> gb(gsz);
    Grad g{};
    CHECK(grad_layout(n, p.nmerges, gb.data(), &g) == gsz);
    CHECK((size_t)((char*)g.gdp - gb.data()) + 8 * nn <= gsz);
    const size_t csz = ckpt_layout(n, (int)p.levels.size(), nullptr, nullptr);
    std::vector<char> cb(csz);
    Ckpt c{};
    CHECK(ckpt_layout(n, (int)p.levels.size(), cb.data(), &c) == csz);
    CHECK((size_t)((char*)c.org - cb.data()) + 4 * nn * p.levels.size() <= csz);
}

static int mode_plan() {
    std::mt19937_64 rng(2605);
    const int leaves[] = {1, 2, 3, 8, 31, 32, 64};
    for (int t = 0; t < 400; ++t) {
        const int B = 1 + (int)(rng() % 12);
        std::vector<long long> offs{0};
        for (int b = 0; b < B; ++b) {
            const int kind = (int)(rng() % 4);
            const long long sz = kind == 0 ? (long long)(rng() % 3) : kind == 1 ? (long long)(rng() % 70)
                               : kind == 2 ? (long long)(rng() % 2000) : (long long)(rng() % 20000);
            offs.push_back(offs.back() + sz);
        }
        check_plan(offs, leaves[t % 7], (t & 1) != 0);
        if (g_fail) return 1;
    }
    check_plan({0, 262144}, 8, false);
    check_plan({0, 65536}, 64, true);
    check_plan({0}, 8, false);
    check_plan({0, 0, 0}, 8, false);
    std::printf("plan ok\n");
    return g_fail ? 1 : 0;
}

static int mode_leaf() {
    int n;
    if (std::scanf("%d", &n) != 1 || n < 1 || n > kLeafMax) return 2;
    std::vector<double> d((size_t)n), e((size_t)n, 0.0), r0((size_t)n), r1((size_t)n);
    for (int i = 0; i < n; ++i)
        if (std::scanf("%lf", &d[(size_t)i]) != 1) return 2;
    for (int i = 0; i + 1 < n; ++i)
        if (std::scanf("%lf", &e[(size_t)i]) != 1) return 2;
    unsigned nrot = 0;
    const int st = leaf_ql(n, d.data(), e.data(), r0.data(), r1.data(), 1, &nrot, 0, n - 1);
    std::printf("%d %u\n", st, nrot);
    for (int i = 0; i < n; ++i) std::printf("%.17g %.17g %.17g\n", d[(size_t)i], r0[(size_t)i], r1[(size_t)i]);
    return 0;
}

static void check_search(const std::vector<double>& v, double x) {
    const int n = (int)v.size();
    int lt = 0, le = 0;
    for (double y : v) {
        lt += (y < x) ? 1 : 0;
        le += (y <= x) ? 1 : 0;
    }
    CHECK(count_lt<false>(v.data(), n, x) == lt);
    CHECK(count_lt<true>(v.data(), n, x) == lt);
    CHECK(count_le<false>(v.data(), n, x) == le);
    CHECK(count_le<true>(v.data(), n, x) == le);
    // the same values as roots: origin og[i] into a shuffled pole list, tau 0
    std::vector<double> poles(v.rbegin(), v.rend());
    std::vector<int> og((size_t)n);
    std::vector<double> tau((size_t)n, 0.0);
    for (int i = 0; i < n; ++i) og[(size_t)i] = n - 1 - i;
    CHECK(roots_cmp_count<false>(poles.data(), og.data(), tau.data(), n, x) == le);
    CHECK(roots_cmp_count<true>(poles.data(), og.data(), tau.data(), n, x) == le);
}

static int mode_search() {
    std::mt19937_64 rng(7);
    for (int t = 0; t < 3000 && !g_fail; ++t) {
        const int n = t < 200 ? t % 40 : (int)(rng() % (t < 2900 ? 3000 : 70000));
        const int span = 1 + (int)(rng() % (n / 2 + 2));  // repeated values when span < n
        std::vector<double> v((size_t)n);
        for (auto& y : v) y = (double)(rng() % (unsigned)span);
        std::sort(v.begin(), v.end());
        for (int q = 0; q < 24 && !g_fail; ++q) {
            const double x = (double)((long long)(rng() % (unsigned)(span + 2)) - 1) + ((q & 1) ? 0.5 : 0.0);
            check_search(v, x);
        }
        if (n > 0 && !g_fail) {
            check_search(v, v.front());
            check_search(v, v.back());
        }
    }
    if (g_fail) return 1;
    std::printf("search ok\n");
    return 0;
}

int main(int argc, char** argv) {
    if (argc > 1 && !std::strcmp(argv[1], "plan")) return mode_plan();
    if (argc > 1 && !std::strcmp(argv[1], "leaf")) return mode_leaf();
    if (argc > 1 && !std::strcmp(argv[1], "search")) return mode_search();
    std::fprintf(stderr, "usage: host_check plan|leaf|search\n");
    return 2;
}
