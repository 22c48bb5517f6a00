// Host-side planning of a solve: the merge-tree tables every launch reads
// and the carving of the caller's workspace, checkpoint and reverse-pass
// scratch.  Plain C++ with no HIP calls, so it also builds (and runs under
// the address and undefined-behaviour sanitizers) on a machine with no GPU.
#include <algorithm>
#include <vector>

#include "tde_plan.h"
#include "tde_tree.h"

namespace tde {

// In-wave merge trees of every leaf size 1..kLeafMax (leaf-local offsets): the
// part of the single-column tree below a leaf, levelled by height.
void sub_trees(std::vector<SubHdr>* hdr, std::vector<SubMerge>* mer) {
    hdr->assign(kLeafMax + 1, SubHdr{});
    mer->clear();
    for (int l = 1; l <= kLeafMax; ++l) {
        const LevelTables t = build_tree(1, {0, (long long)l});
        SubHdr& h = (*hdr)[l];
        h.mbase = (int)mer->size();
        h.H = (int)t.mstart.size();
        for (int k = 0; k < h.H; ++k) h.lv[k] = (unsigned char)t.mstart[k];
        h.lv[h.H] = (unsigned char)t.merges.size();
        for (const MergeRec& R : t.merges)
            mer->push_back(SubMerge{(unsigned char)R.off, (unsigned char)R.nL, (unsigned char)R.nR, (unsigned char)R.pk});
    }
}

int plan_host(Plan* p) {
    const LevelTables t = build_tree(p->leaf, p->offs);
    p->B = (int)p->offs.size() - 1;
    p->ntot = p->offs.back();
    p->levels.clear();
    p->h_blkm.clear();
    int maxM = 1;
    long long maxN = 1;
    for (size_t h = 0; h < t.mstart.size(); ++h) {
        LevelInfo info{};
        info.mstart = t.mstart[h];
        info.M = t.mcount[h];
        info.N = t.ncols[h];
        info.smax = t.smax[h];
        // blkm[b] = merge holding packed column min(b*kWG, N-1), b = 0..nb
        info.bstart = (int)p->h_blkm.size();
        const long long nb = (info.N + kWG - 1) / kWG;
        int m = 0;
        for (long long b = 0; b <= nb; ++b) {
            const long long c = std::min(b * (long long)kWG, info.N - 1);
            while (m + 1 < info.M && t.merges[info.mstart + m + 1].pk <= c) ++m;
            p->h_blkm.push_back(m);
        }
        // in-wave packs: consecutive merges, at most kLeafMax columns per pack
        info.wpstart = (int)p->h_blkm.size();
        info.nwp = 0;
        if (info.smax <= kLeafMax) {
            int cols = 0;
            for (int j = 0; j < info.M; ++j) {
                const MergeRec& R = t.merges[info.mstart + j];
                const int s = R.nL + R.nR;
                if (j == 0 || cols + s > kLeafMax) {
                    p->h_blkm.push_back(j);
                    ++info.nwp;
                    cols = 0;
                }
                cols += s;
            }
            p->h_blkm.push_back(info.M);
        }
        info.all_root = 1;
        for (int j = 0; j < info.M; ++j)
            if (!(t.merges[info.mstart + j].flags & MF_ROOT)) info.all_root = 0;
        maxM = std::max(maxM, info.M);
        maxN = std::max(maxN, info.N);
        p->levels.push_back(info);
    }
    if ((int)p->levels.size() > kMaxLevels) return -1;
    p->maxM = maxM;
    p->maxN = maxN;
    p->h_merges = t.merges;
    p->nmerges = (int)t.merges.size();
    p->h_leaves = t.leaves;
    p->nleaves = (int)t.leaves.size();
    int lmax = 1;
    for (const LeafRec& L : t.leaves) lmax = std::max(lmax, L.size);
    p->leafmax = lmax;
    p->h_shdr.clear();
    p->h_smer.clear();
    if (p->leaf_dc) sub_trees(&p->h_shdr, &p->h_smer);
    return 0;
}

// ---------------------------------------------------------------------------
// Workspace layout (all slices 256-byte aligned)
// ---------------------------------------------------------------------------
size_t workspace_layout(long long n, long long B, long long maxM, char* base, Work* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const long long nn = n > 0 ? n : 1;
    const long long nb = (nn + kWG - 1) / kWG + 2;
    Work t{};
    t.status = (int*)take(kCntOffset);
    t.ticket = t.status ? (unsigned*)((char*)t.status + 16) : nullptr;
    t.counters = (unsigned long long*)take(sizeof(unsigned long long) * CNT_N * kCntSlots);
    t.pmax = (unsigned long long*)take(sizeof(unsigned long long) * (B > 0 ? B : 1));
    t.lam = (double*)take(8 * nn);
    t.blo = (double*)take(8 * nn);
    t.bhi = (double*)take(8 * nn);
    t.D = (double*)take(8 * nn);
    t.Z = (double*)take(8 * nn);
    t.RL = (double*)take(8 * nn);
    t.RH = (double*)take(8 * nn);
    t.src = (int*)take(4 * nn);
    t.D2 = (double*)take(8 * nn);
    t.Z2 = (double*)take(8 * nn);
    t.RL2 = (double*)take(8 * nn);
    t.RH2 = (double*)take(8 * nn);
    t.st = (int*)take(4 * nn);
    // prefix arrays: n + 1 entries for the level-wide scans, plus one per merge
    // (at most n/2 + 1) for k_level_block's merge-local counts
    t.scan = (int*)take(4 * (nn + nn / 2 + 2));
    t.scanC = (int*)take(4 * (nn + nn / 2 + 2));
    t.scanR = (int*)take(4 * (nn + nn / 2 + 2));
    t.bsum = (int*)take(4 * nb);
    t.bcnt = (int*)take(4 * (size_t)kMaxLevels * 2 * nb);
    t.bsumA = t.bcnt;
    t.bsumR = t.bcnt ? t.bcnt + nb : nullptr;
    t.bsumAs = (int*)take(4 * nb);
    t.bsumRs = (int*)take(4 * nb);
    t.nnpos = (int*)take(4 * nn);
    t.cf = (int*)take(4 * nn);
    t.Da = (double*)take(8 * nn);
    t.Za = (double*)take(8 * nn);
    t.Wa = (double*)take(8 * nn);
    t.RLa = (double*)take(8 * nn);
    t.RHa = (double*)take(8 * nn);
    t.amerge = (int*)take(4 * nn);
    t.witems = (int*)take(4 * (nn + 2));
    t.apos = (int*)take(4 * nn);
    t.rpos = (int*)take(4 * nn);
    t.dpos = (int*)take(4 * nn);
    t.org = (int*)take(4 * nn);
    t.tau = (double*)take(8 * nn);
    t.rootval = (double*)take(8 * nn);
    t.dorg = (double*)take(8 * nn);
    t.zhat = (double*)take(8 * nn);
    t.PBL = (double*)take(8 * nn);
    t.PBH = (double*)take(8 * nn);
    t.Dd = (double*)take(8 * nn);
    t.RLd = (double*)take(8 * nn);
    t.RHd = (double*)take(8 * nn);
    t.Dr = (double*)take(8 * nn);
    t.RLr = (double*)take(8 * nn);
    t.RHr = (double*)take(8 * nn);
    t.sec_cap = kSecMaxIter;
    (void)maxM;
    if (w) *w = t;
    return off;
}

size_t grad_layout(long long n, long long nmerges, char* base, Grad* g) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const long long nn = n > 0 ? n : 1;
    Grad t{};
    t.glam = (double*)take(8 * nn);
    t.gblo = (double*)take(8 * nn);
    t.gbhi = (double*)take(8 * nn);
    t.gD = (double*)take(8 * nn);
    t.gZ = (double*)take(8 * nn);
    t.gRL = (double*)take(8 * nn);
    t.gRH = (double*)take(8 * nn);
    t.gD2 = (double*)take(8 * nn);
    t.gZ2 = (double*)take(8 * nn);
    t.gRL2 = (double*)take(8 * nn);
    t.gRH2 = (double*)take(8 * nn);
    t.glr = (double*)take(8 * nn);
    t.gbr = (double*)take(8 * nn);
    t.ghr = (double*)take(8 * nn);
    t.coef = (double*)take(8 * 10 * nn);
    t.chain = (RunState*)take(sizeof(RunState) * nn);
    t.cdef = (RunState*)take(sizeof(RunState) * nn);
    t.skey = (double*)take(8 * nn);
    t.sidx = (int*)take(4 * nn);
    t.grho = (double*)take(8 * (nmerges > 0 ? nmerges : 1));
    t.gdp = (double*)take(8 * nn);
    if (g) *g = t;
    return off;
}

size_t ckpt_layout(long long n, int levels, char* base, Ckpt* c) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const long long nn = n > 0 ? n : 1;
    const long long H = levels > 0 ? levels : 0;
    Ckpt t{};
    t.n = nn;
    (void)take(256);  // header slot: the size is never 0, even for a tree with no merges
    t.lam = (double*)take(8 * nn * H);
    t.blo = (double*)take(8 * nn * H);
    t.bhi = (double*)take(8 * nn * H);
    t.tau = (double*)take(8 * nn * H);
    t.org = (int*)take(4 * nn * H);
    if (c) *c = t;
    return off;
}

}  // namespace tde
