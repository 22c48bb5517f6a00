// Static D&C tree of a batch of problems (host only): balanced halving
// (split at floor(size/2)) down to leaves of at most `leaf` columns, merges
// levelled by height so that both children of a merge are complete before
// it runs (the level-by-level schedule of Section 4.1, across all problems).
#pragma once
#include <algorithm>
#include <vector>

#include "tde_internal.h"

namespace tde {

struct LevelTables {
    std::vector<MergeRec> merges;   // flat, level after level, ascending off within a level
    std::vector<int> mstart;        // first merge of each level
    std::vector<int> mcount;        // merges per level
    std::vector<long long> ncols;   // packed columns per level
    std::vector<int> smax;          // largest merge per level
    std::vector<LeafRec> leaves;
};

namespace detail {
struct TreeBuilder {
    int leaf;
    std::vector<std::vector<MergeRec>> lv;
    std::vector<LeafRec> leaves;

    int build(long long off, long long size, int prob, long long pstart, long long pend) {
        if (size <= leaf) {
            LeafRec L{};
            L.off = off;
            L.size = (int)size;
            L.prob = prob;
            L.flags = (off > pstart ? LF_TEAR_LEFT : 0) | (off + size < pend ? LF_TEAR_RIGHT : 0) |
                      (size == pend - pstart ? LF_WHOLE : 0);
            leaves.push_back(L);
            return 0;
        }
        const long long nL = size / 2, nR = size - nL;
        const int hL = build(off, nL, prob, pstart, pend);
        const int hR = build(off + nL, nR, prob, pstart, pend);
        const int h = std::max(hL, hR) + 1;
        if ((int)lv.size() < h) lv.resize(h);
        MergeRec R{};
        R.off = off;
        R.nL = (int)nL;
        R.nR = (int)nR;
        R.prob = prob;
        R.flags = (size == pend - pstart) ? MF_ROOT : 0;
        lv[h - 1].push_back(R);
        return h;
    }
};
}  // namespace detail

inline LevelTables build_tree(int leaf, const std::vector<long long>& offs) {
    detail::TreeBuilder tb;
    tb.leaf = leaf;
    const int B = (int)offs.size() - 1;
    for (int b = 0; b < B; ++b) {
        const long long lo = offs[b], hi = offs[b + 1];
        if (hi > lo) tb.build(lo, hi - lo, b, lo, hi);
    }
    LevelTables t;
    for (auto& L : tb.lv) {
        std::sort(L.begin(), L.end(), [](const MergeRec& a, const MergeRec& b) { return a.off < b.off; });
        t.mstart.push_back((int)t.merges.size());
        t.mcount.push_back((int)L.size());
        long long pk = 0;
        int sm = 0;
        for (auto& R : L) {
            R.pk = pk;
            pk += R.nL + R.nR;
            sm = std::max(sm, R.nL + R.nR);
            t.merges.push_back(R);
        }
        t.ncols.push_back(pk);
        t.smax.push_back(sm);
    }
    t.leaves = std::move(tb.leaves);
    return t;
}

}  // namespace tde
