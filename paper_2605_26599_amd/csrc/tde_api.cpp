// C-ABI of the BR D&C eigenvalue library: argument checks, plan cache and
// workspace carving.  The numerical work is enqueued by enqueue_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/tde.h"
#include "tde_plan.h"
#include "tde_tree.h"

namespace tde {
namespace {

using PlanKey = std::tuple<int, int, int, int, bool, std::vector<long long>>;
std::mutex g_mu;
std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

// Captured passes: one executable graph per (plan, pass kind, buffers).
// Capture runs on an internal stream per device; replays run on the
// caller's stream.
enum { PASS_SOLVE = 0, PASS_CKPT = 1, PASS_BACKWARD = 2, PASS_ROWS = 3 };
using Bufs = std::array<const void*, 8>;
using GraphKey = std::tuple<const Plan*, int, Bufs>;
std::map<GraphKey, hipGraphExec_t> g_graphs;
std::map<int, hipStream_t> g_capture_streams;
constexpr size_t kMaxGraphs = 64;

void drop_graphs() {
    for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
}

int graph_for(const Plan& plan, int kind, const Bufs& bufs, const std::function<int(void*)>& enqueue,
              hipGraphExec_t* exec) {
    GraphKey key{&plan, kind, bufs};
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        *exec = it->second;
        return TDE_OK;
    }
    if (g_graphs.size() >= kMaxGraphs) drop_graphs();
    hipStream_t cs;
    auto sit = g_capture_streams.find(plan.device);
    if (sit == g_capture_streams.end()) {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return TDE_EDEVICE;
        g_capture_streams[plan.device] = cs;
    } else {
        cs = sit->second;
    }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return TDE_EDEVICE;
    const int rc = enqueue(cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != 0 || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return TDE_EDEVICE;
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return TDE_EDEVICE;
    g_graphs.emplace(key, ge);
    *exec = ge;
    return TDE_OK;
}

// Runs enqueue either eagerly on the caller's stream or through the graph
// cache, as the options and timing mode ask.
int run_pass(const Plan& plan, int kind, const Bufs& bufs, const tde_opts* opts, void* stream,
             const std::function<int(void*)>& enqueue) {
    const bool use_graph = !(opts && (opts->flags & TDE_FLAG_NO_GRAPH)) && !timing_enabled();
    if (use_graph) {
        hipGraphExec_t ge = nullptr;
        int rc;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            rc = graph_for(plan, kind, bufs, enqueue, &ge);
        }
        if (rc != TDE_OK) return rc;
        return hipGraphLaunch(ge, (hipStream_t)stream) == hipSuccess ? TDE_OK : TDE_EDEVICE;
    }
    return enqueue(stream) == 0 ? TDE_OK : TDE_EDEVICE;
}

void free_plan(Plan* p) {
    if (p->d_merges) (void)hipFree(p->d_merges);
    if (p->d_leaves) (void)hipFree(p->d_leaves);
    if (p->d_offs) (void)hipFree(p->d_offs);
    if (p->d_blkm) (void)hipFree(p->d_blkm);
    if (p->d_shdr) (void)hipFree(p->d_shdr);
    if (p->d_smer) (void)hipFree(p->d_smer);
    p->d_shdr = nullptr;
    p->d_smer = nullptr;
    p->d_blkm = nullptr;
    p->d_merges = nullptr;
    p->d_leaves = nullptr;
    p->d_offs = nullptr;
}

// In-wave merge trees of every leaf size 1..kLeafMax (leaf-local offsets).
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

int make_plan(int device, int leaf, int cols, int wmin, bool dc, const std::vector<long long>& offs, Plan** out) {
    PlanKey key{device, leaf, cols, wmin, dc, offs};
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return TDE_OK;
    }
    auto p = std::make_unique<Plan>();
    p->device = device;
    p->leaf = leaf;
    p->sweep_cols = cols;
    p->wide_min = wmin;
    p->leaf_dc = dc;
    p->offs = offs;
    p->B = (int)offs.size() - 1;
    p->ntot = offs.back();
    const LevelTables t = build_tree(leaf, offs);
    const std::vector<MergeRec>& flat = t.merges;
    int maxM = 1;
    long long maxN = 1;
    std::vector<int> blkm;
    for (size_t h = 0; h < t.mstart.size(); ++h) {
        LevelInfo info{};
        info.mstart = t.mstart[h];
        info.M = t.mcount[h];
        info.N = t.ncols[h];
        info.smax = t.smax[h];
        // blkm[b] = merge holding packed column min(b*kWG, N-1), b = 0..nb
        info.bstart = (int)blkm.size();
        const long long nb = (info.N + kWG - 1) / kWG;
        int m = 0;
        for (long long b = 0; b <= nb; ++b) {
            const long long c = std::min(b * (long long)kWG, info.N - 1);
            while (m + 1 < info.M && flat[info.mstart + m + 1].pk <= c) ++m;
            blkm.push_back(m);
        }
        maxM = std::max(maxM, info.M);
        maxN = std::max(maxN, info.N);
        p->levels.push_back(info);
    }
    p->maxM = maxM;
    p->maxN = maxN;
    p->nmerges = (int)flat.size();
    if ((int)p->levels.size() > kMaxLevels) return TDE_EINVAL;
    p->nleaves = (int)t.leaves.size();
    int lmax = 1;
    for (auto& L : t.leaves) lmax = std::max(lmax, L.size);
    p->leafmax = lmax;
    auto upload = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (bytes == 0) bytes = 8;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
        return true;
    };
    bool ok = upload((void**)&p->d_merges, flat.empty() ? nullptr : flat.data(), flat.size() * sizeof(MergeRec)) &&
              upload((void**)&p->d_leaves, t.leaves.empty() ? nullptr : t.leaves.data(),
                     t.leaves.size() * sizeof(LeafRec)) &&
              upload((void**)&p->d_offs, offs.data(), offs.size() * sizeof(long long)) &&
              upload((void**)&p->d_blkm, blkm.empty() ? nullptr : blkm.data(), blkm.size() * sizeof(int));
    if (ok && dc) {
        std::vector<SubHdr> sh;
        std::vector<SubMerge> sm;
        sub_trees(&sh, &sm);
        ok = upload((void**)&p->d_shdr, sh.data(), sh.size() * sizeof(SubHdr)) &&
             upload((void**)&p->d_smer, sm.data(), sm.size() * sizeof(SubMerge));
    }
    if (!ok) {
        free_plan(p.get());
        return TDE_ENOMEM;
    }
    *out = p.get();
    g_plans.emplace(std::move(key), std::move(p));
    return TDE_OK;
}

int resolve_opts(const tde_opts* opts, int* leaf, int* cols, int* wmin = nullptr, bool* dc = nullptr) {
    int L = kDefaultLeaf, C = kDefaultSweepCols, W = kWideMin;
    if (opts) {
        if (opts->flags & ~(TDE_FLAG_NO_GRAPH | TDE_FLAG_LEAF_DC)) return TDE_EINVAL;
        if (opts->leaf != 0) L = opts->leaf;
        if (opts->sweep_cols != 0) C = opts->sweep_cols;
        if (opts->wide_min != 0) W = opts->wide_min;
    }
    if (L < 1 || L > kLeafMax) return TDE_EINVAL;
    if (C < 1 || C > (1 << 20)) return TDE_EINVAL;
    if (W < 2) return TDE_EINVAL;
    *leaf = L;
    *cols = C;
    if (wmin) *wmin = W;
    if (dc) *dc = opts && (opts->flags & TDE_FLAG_LEAF_DC);
    return TDE_OK;
}

// Tree height of the largest problem (levels of the plan), host only.
int tree_levels(int leaf, const std::vector<long long>& offs) {
    int H = 0;
    for (size_t b = 0; b + 1 < offs.size(); ++b) {
        long long sz = offs[b + 1] - offs[b];
        int h = 0;
        while (sz > leaf) {
            sz -= sz / 2;  // the larger child (balanced halving)
            ++h;
        }
        H = std::max(H, h);
    }
    return H;
}

int check_offsets(const int64_t* offsets, int64_t B, std::vector<long long>* offs) {
    if (B < 0 || (B > 0 && !offsets)) return TDE_EINVAL;
    offs->assign((size_t)B + 1, 0);
    for (int64_t b = 0; b <= B && B > 0; ++b) (*offs)[b] = offsets[b];
    if (B > 0 && (*offs)[0] != 0) return TDE_EINVAL;
    for (int64_t b = 0; b < B; ++b)
        if ((*offs)[b + 1] < (*offs)[b]) return TDE_EINVAL;
    if ((*offs)[B] > (long long)0x3fffffff) return TDE_EINVAL;
    return TDE_OK;
}

int get_plan(const tde_opts* opts, const std::vector<long long>& offs, Plan** plan) {
    int leaf, cols, wmin;
    bool dc;
    if (resolve_opts(opts, &leaf, &cols, &wmin, &dc) != TDE_OK) return TDE_EINVAL;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return TDE_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    return make_plan(device, leaf, cols, wmin, dc, offs, plan);
}

bool needs_e(const std::vector<long long>& offs) {
    for (size_t b = 0; b + 1 < offs.size(); ++b)
        if (offs[b + 1] - offs[b] > 1) return true;
    return false;
}

int solve(const double* d, const double* e, const std::vector<long long>& offs, double* lambda, void* ws,
          size_t ws_bytes, void* stream, const tde_opts* opts, void* ckpt = nullptr, size_t ckpt_bytes = 0,
          double* qfirst = nullptr, double* qlast = nullptr) {
    int leaf, cols;
    if (resolve_opts(opts, &leaf, &cols) != TDE_OK) return TDE_EINVAL;
    const long long ntot = offs.back();
    const long long B = (long long)offs.size() - 1;
    if (ntot == 0) return TDE_OK;
    if (!d || !lambda || !ws) return TDE_EINVAL;
    if (needs_e(offs) && !e) return TDE_EINVAL;
    if (ws_bytes < workspace_layout(ntot, B, ntot, nullptr, nullptr)) return TDE_EINVAL;
    const int H = tree_levels(leaf, offs);
    if (ckpt_bytes && (!ckpt || ckpt_bytes < ckpt_layout(ntot, H, nullptr, nullptr))) return TDE_EINVAL;
    Plan* plan = nullptr;
    int rc = get_plan(opts, offs, &plan);
    if (rc != TDE_OK) return rc;
    Work w{};
    workspace_layout(ntot, B, ntot, (char*)ws, &w);
    if (qfirst || qlast) {
        w.qfirst = qfirst;
        w.qlast = qlast;
        w.rows_out = 1;
        Bufs bufs{d, e, lambda, ws, qfirst, qlast, nullptr, nullptr};
        return run_pass(*plan, PASS_ROWS, bufs, opts, stream,
                        [&](void* s) { return enqueue_solve(*plan, w, d, e, lambda, s); });
    }
    if (!ckpt_bytes) {
        Bufs bufs{d, e, lambda, ws, nullptr, nullptr, nullptr, nullptr};
        return run_pass(*plan, PASS_SOLVE, bufs, opts, stream,
                        [&](void* s) { return enqueue_solve(*plan, w, d, e, lambda, s); });
    }
    Ckpt ck{};
    ckpt_layout(ntot, (int)plan->levels.size(), (char*)ckpt, &ck);
    Bufs bufs{d, e, lambda, ws, ckpt, nullptr, nullptr, nullptr};
    return run_pass(*plan, PASS_CKPT, bufs, opts, stream,
                    [&](void* s) { return enqueue_solve(*plan, w, d, e, lambda, s, &ck); });
}

int backward(const double* d, const double* e, const std::vector<long long>& offs, const double* gin,
             const void* ckpt, size_t ckpt_bytes, double* gd, double* ge, void* ws, size_t ws_bytes, void* stream,
             const tde_opts* opts) {
    int leaf, cols;
    if (resolve_opts(opts, &leaf, &cols) != TDE_OK) return TDE_EINVAL;
    const long long ntot = offs.back();
    const long long B = (long long)offs.size() - 1;
    if (ntot == 0) return TDE_OK;
    if (!d || !gin || !ckpt || !gd || !ge || !ws) return TDE_EINVAL;
    if (needs_e(offs) && !e) return TDE_EINVAL;
    const int H = tree_levels(leaf, offs);
    if (ckpt_bytes < ckpt_layout(ntot, H, nullptr, nullptr)) return TDE_EINVAL;
    const size_t fw = workspace_layout(ntot, B, ntot, nullptr, nullptr);
    Plan* plan = nullptr;
    int rc = get_plan(opts, offs, &plan);
    if (rc != TDE_OK) return rc;
    if (ws_bytes < fw + grad_layout(ntot, ntot, nullptr, nullptr)) return TDE_EINVAL;
    Work w{};
    workspace_layout(ntot, B, ntot, (char*)ws, &w);
    Grad gr{};
    grad_layout(ntot, plan->nmerges, (char*)ws + fw, &gr);
    Ckpt ck{};
    ckpt_layout(ntot, (int)plan->levels.size(), (char*)const_cast<void*>(ckpt), &ck);
    Bufs bufs{d, e, gin, ckpt, gd, ge, ws, nullptr};
    return run_pass(*plan, PASS_BACKWARD, bufs, opts, stream,
                    [&](void* s) { return enqueue_backward(*plan, w, gr, ck, d, e, gin, gd, ge, s); });
}

// Driver pre-pass: pairwise merge schedule of the blocks of every problem
// (balanced over the blocks, levelled by height), cached per split.
struct RunMerges {
    std::vector<std::pair<int, int>> levels;  // (first record, count) per pass
    MergeRec* d_recs = nullptr;
};
using RunKey = std::tuple<int, std::vector<long long>, std::vector<long long>>;
std::map<RunKey, RunMerges> g_runs;
constexpr size_t kMaxRunSchedules = 64;

int run_merge_build(const std::vector<long long>& nb, int bs, int be, std::vector<std::vector<MergeRec>>* lv) {
    if (be - bs <= 1) return 0;
    const int mid = bs + (be - bs) / 2;
    const int h = std::max(run_merge_build(nb, bs, mid, lv), run_merge_build(nb, mid, be, lv)) + 1;
    if ((int)lv->size() < h) lv->resize(h);
    MergeRec R{};
    R.off = nb[bs];
    R.nL = (int)(nb[mid] - nb[bs]);
    R.nR = (int)(nb[be] - nb[mid]);
    (*lv)[h - 1].push_back(R);
    return h;
}

int get_run_merges(int device, const std::vector<long long>& offs, const std::vector<long long>& nb,
                   const RunMerges** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    RunKey key{device, offs, nb};
    auto it = g_runs.find(key);
    if (it != g_runs.end()) {
        *out = &it->second;
        return TDE_OK;
    }
    if (g_runs.size() >= kMaxRunSchedules) {
        for (auto& kv : g_runs)
            if (kv.second.d_recs) (void)hipFree(kv.second.d_recs);
        g_runs.clear();
    }
    std::vector<std::vector<MergeRec>> lv;
    size_t bi = 0;  // first block of problem b
    for (size_t b = 0; b + 1 < offs.size(); ++b) {
        size_t be = bi;
        while (be + 1 < nb.size() && nb[be] < offs[b + 1]) ++be;
        run_merge_build(nb, (int)bi, (int)be, &lv);
        bi = be;
    }
    RunMerges rm;
    std::vector<MergeRec> flat;
    for (auto& L : lv) {
        std::sort(L.begin(), L.end(), [](const MergeRec& a, const MergeRec& b) { return a.off < b.off; });
        rm.levels.emplace_back((int)flat.size(), (int)L.size());
        flat.insert(flat.end(), L.begin(), L.end());
    }
    if (!flat.empty()) {
        if (hipMalloc(&rm.d_recs, flat.size() * sizeof(MergeRec)) != hipSuccess) return TDE_ENOMEM;
        if (hipMemcpy(rm.d_recs, flat.data(), flat.size() * sizeof(MergeRec), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(rm.d_recs);
            return TDE_EDEVICE;
        }
    }
    *out = &g_runs.emplace(std::move(key), std::move(rm)).first->second;
    return TDE_OK;
}

int solve_split(const double* d, const double* e, const std::vector<long long>& offs, double* lambda, void* ws,
                size_t ws_bytes, void* stream, const tde_opts* opts, int64_t* nblocks) {
    int leaf, cols;
    if (resolve_opts(opts, &leaf, &cols) != TDE_OK) return TDE_EINVAL;
    const long long ntot = offs.back();
    if (nblocks) *nblocks = 0;
    if (ntot == 0) return TDE_OK;
    if (!d || !lambda || !ws) return TDE_EINVAL;
    if (needs_e(offs) && !e) return TDE_EINVAL;
    // room for the worst case, every column its own block
    if (ws_bytes < workspace_layout(ntot, ntot, ntot, nullptr, nullptr)) return TDE_EINVAL;
    Work w{};
    workspace_layout(ntot, ntot, ntot, (char*)ws, &w);
    if (enqueue_split_flags(d, e, ntot, w.st, stream) != 0) return TDE_EDEVICE;
    std::vector<int> flags((size_t)ntot);
    if (hipMemcpyAsync(flags.data(), w.st, sizeof(int) * (size_t)ntot, hipMemcpyDeviceToHost,
                       (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return TDE_EDEVICE;
    std::vector<long long> nb;
    for (size_t b = 0; b + 1 < offs.size(); ++b)
        for (long long i = offs[b]; i < offs[b + 1]; ++i)
            if (i == offs[b] || flags[(size_t)i]) nb.push_back(i);
    nb.push_back(ntot);
    if (nblocks) *nblocks = (int64_t)nb.size() - 1;
    int rc = solve(d, e, nb, lambda, ws, ws_bytes, stream, opts);
    if (rc != TDE_OK) return rc;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return TDE_EDEVICE;
    const RunMerges* rm = nullptr;
    rc = get_run_merges(device, offs, nb, &rm);
    if (rc != TDE_OK) return rc;
    if (rm->levels.empty()) return TDE_OK;
    Work ws2{};
    workspace_layout(ntot, (long long)nb.size() - 1, ntot, (char*)ws, &ws2);
    double* src = lambda;
    double* dst = ws2.D;  // free once the solve is done (same stream)
    for (const auto& L : rm->levels) {
        if (enqueue_merge_runs(rm->d_recs + L.first, L.second, src, dst, ntot, stream) != 0) return TDE_EDEVICE;
        std::swap(src, dst);
    }
    if (src != lambda &&
        hipMemcpyAsync(lambda, src, sizeof(double) * (size_t)ntot, hipMemcpyDeviceToDevice, (hipStream_t)stream) !=
            hipSuccess)
        return TDE_EDEVICE;
    return TDE_OK;
}

}  // namespace
}  // namespace tde

extern "C" {

int tde_version(void) { return 200; }

size_t tde_workspace_bytes(int64_t n_total, int64_t batch, const tde_opts* opts) {
    int leaf, cols;
    if (n_total < 0 || batch < 0 || tde::resolve_opts(opts, &leaf, &cols) != TDE_OK) return 0;
    return tde::workspace_layout(n_total, batch, n_total, nullptr, nullptr);
}

int tde_eigvals(const double* d, const double* e, int64_t n, double* lambda, void* ws, size_t ws_bytes,
                void* hip_stream, const tde_opts* opts) {
    if (n < 0 || n > (int64_t)0x3fffffff) return TDE_EINVAL;
    std::vector<long long> offs{0, (long long)n};
    return tde::solve(d, e, offs, lambda, ws, ws_bytes, hip_stream, opts);
}

int tde_eigvals_split(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                      void* ws, size_t ws_bytes, void* hip_stream, const tde_opts* opts, int64_t* nblocks) {
    std::vector<long long> offs;
    if (tde::check_offsets(offsets, B, &offs) != TDE_OK) return TDE_EINVAL;
    return tde::solve_split(d, e, offs, lambda, ws, ws_bytes, hip_stream, opts, nblocks);
}

int tde_eigvals_batched(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                        void* ws, size_t ws_bytes, void* hip_stream, const tde_opts* opts) {
    std::vector<long long> offs;
    if (tde::check_offsets(offsets, B, &offs) != TDE_OK) return TDE_EINVAL;
    if (B == 0) return TDE_OK;
    return tde::solve(d, e, offs, lambda, ws, ws_bytes, hip_stream, opts);
}

int tde_eigvals_rows(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                     double* qfirst, double* qlast, void* ws, size_t ws_bytes, void* hip_stream,
                     const tde_opts* opts) {
    std::vector<long long> offs;
    if (tde::check_offsets(offsets, B, &offs) != TDE_OK) return TDE_EINVAL;
    if (!qfirst && !qlast) return TDE_EINVAL;
    if (B == 0 || offs.back() == 0) return TDE_OK;
    return tde::solve(d, e, offs, lambda, ws, ws_bytes, hip_stream, opts, nullptr, 0, qfirst, qlast);
}

size_t tde_checkpoint_bytes(const int64_t* offsets, int64_t B, const tde_opts* opts) {
    int leaf, cols;
    std::vector<long long> offs;
    if (tde::resolve_opts(opts, &leaf, &cols) != TDE_OK || tde::check_offsets(offsets, B, &offs) != TDE_OK) return 0;
    return tde::ckpt_layout(offs.back(), tde::tree_levels(leaf, offs), nullptr, nullptr);
}

size_t tde_backward_workspace_bytes(int64_t n_total, int64_t batch, const tde_opts* opts) {
    int leaf, cols;
    if (n_total < 0 || batch < 0 || tde::resolve_opts(opts, &leaf, &cols) != TDE_OK) return 0;
    return tde::workspace_layout(n_total, batch, n_total, nullptr, nullptr) +
           tde::grad_layout(n_total, n_total, nullptr, nullptr);
}

int tde_eigvals_ckpt(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                     void* ckpt, size_t ckpt_bytes, void* ws, size_t ws_bytes, void* hip_stream,
                     const tde_opts* opts) {
    std::vector<long long> offs;
    if (tde::check_offsets(offsets, B, &offs) != TDE_OK) return TDE_EINVAL;
    if (B == 0 || offs.back() == 0) return TDE_OK;
    if (!ckpt || ckpt_bytes == 0) return TDE_EINVAL;
    return tde::solve(d, e, offs, lambda, ws, ws_bytes, hip_stream, opts, ckpt, ckpt_bytes);
}

int tde_eigvals_backward(const double* d, const double* e, const int64_t* offsets, int64_t B,
                         const double* glambda, const void* ckpt, size_t ckpt_bytes, double* gd, double* ge,
                         void* ws, size_t ws_bytes, void* hip_stream, const tde_opts* opts) {
    std::vector<long long> offs;
    if (tde::check_offsets(offsets, B, &offs) != TDE_OK) return TDE_EINVAL;
    if (B == 0 || offs.back() == 0) return TDE_OK;
    return tde::backward(d, e, offs, glambda, ckpt, ckpt_bytes, gd, ge, ws, ws_bytes, hip_stream, opts);
}

int tde_get_status(const void* ws, void* hip_stream) {
    if (!ws) return TDE_EINVAL;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return TDE_EDEVICE;
    int st = 0;
    if (hipMemcpy(&st, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return TDE_EDEVICE;
    if (st & tde::ST_NONFINITE) return TDE_ENONFINITE;
    if (st & (tde::ST_LEAF_NOCONV | tde::ST_SEC_NOCONV)) return TDE_ENOCONV;
    return TDE_OK;
}

int tde_get_counters(const void* ws, void* hip_stream, uint64_t* out, int n) {
    if (!ws || !out || n < 0) return TDE_EINVAL;
    if (n > tde::CNT_N) n = tde::CNT_N;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return TDE_EDEVICE;
    if (n == 0) return TDE_OK;
    std::vector<uint64_t> slots((size_t)n * tde::kCntSlots);
    if (hipMemcpy(slots.data(), (const char*)ws + tde::kCntOffset, sizeof(uint64_t) * slots.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return TDE_EDEVICE;
    for (int c = 0; c < n; ++c) {
        uint64_t v = 0;
        for (int k = 0; k < tde::kCntSlots; ++k) v += slots[(size_t)c * tde::kCntSlots + k];
        out[c] = v;
    }
    return TDE_OK;
}

int tde_timing_enable(int on) {
    tde::timing_enable(on != 0);
    return TDE_OK;
}

int tde_timing_read(double* ms, int64_t* launches, int nkinds) {
    if (!ms || !launches || nkinds < 0) return TDE_EINVAL;
    std::vector<long long> cnt(nkinds > 0 ? nkinds : 1);
    int rc = tde::timing_read(ms, cnt.data(), nkinds);
    for (int k = 0; k < nkinds; ++k) launches[k] = cnt[k];
    return rc == 0 ? TDE_OK : TDE_EDEVICE;
}

void tde_release_plans(void) {
    std::lock_guard<std::mutex> lk(tde::g_mu);
    tde::drop_graphs();
    for (auto& kv : tde::g_plans) tde::free_plan(kv.second.get());
    tde::g_plans.clear();
    for (auto& kv : tde::g_runs)
        if (kv.second.d_recs) (void)hipFree(kv.second.d_recs);
    tde::g_runs.clear();
}

const char* tde_status_string(int status) {
    switch (status) {
        case TDE_OK: return "ok";
        case TDE_EINVAL: return "invalid argument";
        case TDE_ENOMEM: return "out of memory";
        case TDE_EDEVICE: return "HIP runtime error";
        case TDE_ENONFINITE: return "non-finite input";
        case TDE_ENOCONV: return "iteration did not converge";
        default: return "unknown status";
    }
}

}  // extern "C"
