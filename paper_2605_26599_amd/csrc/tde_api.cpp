// C-ABI of the BR D&C eigenvalue library: argument checks, plan cache and
// workspace carving.  The numerical work is enqueued by enqueue_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <functional>
#include <iterator>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/tde.h"
#include "tde_dense.h"
#include "tde_plan.h"
#include "tde_tree.h"

namespace tde {
namespace {

// ---------------------------------------------------------------------------
// Caches.  One (recursive) mutex guards them all; every entry point holds it
// from the plan lookup to the last launch it enqueues, so no other thread can
// evict a plan or an executable graph that a call is still using.
//
// Plans: bounded, least recently used first out.  Graph executables: bounded,
// least recently used first out; an event recorded after every launch of an
// executable is waited for before it is destroyed, so an executable still
// queued on a caller's stream is never freed.  Evicting a plan first drops its
// graphs, then waits for the device before freeing its tables (eager launches
// may still read them).
// ---------------------------------------------------------------------------
std::recursive_mutex g_mu;

using PlanKey = std::tuple<int, int, int, int, bool, int, int, int, std::vector<long long>>;
constexpr size_t kMaxPlans = 32;
struct PlanEntry {
    PlanKey key;
    std::unique_ptr<Plan> plan;
};
std::list<PlanEntry> g_plan_lru;  // front = most recently used
std::map<PlanKey, std::list<PlanEntry>::iterator> g_plans;

// Captured passes: one executable graph per (plan, pass kind, buffers).
// Capture runs on an internal stream per device; replays run on the
// caller's stream.
enum { PASS_SOLVE = 0, PASS_CKPT = 1, PASS_BACKWARD = 2, PASS_ROWS = 3, PASS_DENSE = 4 };
using Bufs = std::array<const void*, 8>;
using GraphKey = std::tuple<const Plan*, int, Bufs>;
constexpr size_t kMaxGraphs = 64;
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    hipEvent_t done;  // recorded after every launch of exec
    int device;
};
std::list<GraphEntry> g_graph_lru;  // front = most recently used
std::map<GraphKey, std::list<GraphEntry>::iterator> g_graphs;
std::map<int, hipStream_t> g_capture_streams;

// Scoped switch to another device (restored on exit).
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

void destroy_graph(GraphEntry& ge) {
    DeviceScope ds(ge.device);
    (void)hipEventSynchronize(ge.done);  // the last launch has finished
    (void)hipGraphExecDestroy(ge.exec);
    (void)hipEventDestroy(ge.done);
}

void drop_graphs_if(const std::function<bool(const GraphEntry&)>& pred) {
    for (auto it = g_graph_lru.begin(); it != g_graph_lru.end();) {
        if (pred(*it)) {
            destroy_graph(*it);
            g_graphs.erase(it->key);
            it = g_graph_lru.erase(it);
        } else {
            ++it;
        }
    }
}

void free_plan(Plan* p) {
    DeviceScope ds(p->device);
    (void)hipDeviceSynchronize();  // eager launches may still read the tables
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

void evict_plan(std::list<PlanEntry>::iterator it) {
    const Plan* p = it->plan.get();
    drop_graphs_if([p](const GraphEntry& g) { return std::get<0>(g.key) == p; });
    free_plan(it->plan.get());
    g_plans.erase(it->key);
    g_plan_lru.erase(it);
}

// Caller holds g_mu.
int graph_for(const Plan& plan, int kind, const Bufs& bufs, const std::function<int(void*)>& enqueue,
              GraphEntry** out) {
    GraphKey key{&plan, kind, bufs};
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        g_graph_lru.splice(g_graph_lru.begin(), g_graph_lru, it->second);
        *out = &*it->second;
        return TDE_OK;
    }
    if (g_graph_lru.size() >= kMaxGraphs) {  // least recently used out
        auto last = std::prev(g_graph_lru.end());
        destroy_graph(*last);
        g_graphs.erase(last->key);
        g_graph_lru.erase(last);
    }
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
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(ge);
        return TDE_EDEVICE;
    }
    g_graph_lru.push_front(GraphEntry{key, ge, ev, plan.device});
    g_graphs.emplace(key, g_graph_lru.begin());
    *out = &g_graph_lru.front();
    return TDE_OK;
}

// Runs enqueue either eagerly on the caller's stream or through the graph
// cache, as the options and timing mode ask.
int run_pass(const Plan& plan, int kind, const Bufs& bufs, const tde_opts* opts, void* stream,
             const std::function<int(void*)>& enqueue) {
    const bool use_graph = !(opts && (opts->flags & TDE_FLAG_NO_GRAPH)) && !timing_enabled();
    if (use_graph) {
        GraphEntry* ge = nullptr;
        const int rc = graph_for(plan, kind, bufs, enqueue, &ge);
        if (rc != TDE_OK) return rc;
        if (hipGraphLaunch(ge->exec, (hipStream_t)stream) != hipSuccess) return TDE_EDEVICE;
        return hipEventRecord(ge->done, (hipStream_t)stream) == hipSuccess ? TDE_OK : TDE_EDEVICE;
    }
    return enqueue(stream) == 0 ? TDE_OK : TDE_EDEVICE;
}

// Caller holds g_mu.
int make_plan(int device, int leaf, int cols, int wmin, bool dc, int gmax, int wblocks, int ffew,
              const std::vector<long long>& offs, Plan** out) {
    PlanKey key{device, leaf, cols, wmin, dc, gmax, wblocks, ffew, offs};
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        g_plan_lru.splice(g_plan_lru.begin(), g_plan_lru, it->second);
        *out = it->second->plan.get();
        return TDE_OK;
    }
    auto p = std::make_unique<Plan>();
    p->device = device;
    p->leaf = leaf;
    p->sweep_cols = cols;
    p->wide_min = wmin;
    p->leaf_dc = dc;
    p->group_max = gmax;
    p->wide_blocks = wblocks;
    p->fuse_few = ffew;
    p->offs = offs;
    if (plan_host(p.get()) != 0) return TDE_EINVAL;
    auto upload = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (bytes == 0) bytes = 8;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
        return true;
    };
    auto vec = [](const auto& v) -> const void* { return v.empty() ? nullptr : (const void*)v.data(); };
    bool ok = upload((void**)&p->d_merges, vec(p->h_merges), p->h_merges.size() * sizeof(MergeRec)) &&
              upload((void**)&p->d_leaves, vec(p->h_leaves), p->h_leaves.size() * sizeof(LeafRec)) &&
              upload((void**)&p->d_offs, offs.data(), offs.size() * sizeof(long long)) &&
              upload((void**)&p->d_blkm, vec(p->h_blkm), p->h_blkm.size() * sizeof(int));
    if (ok && dc)
        ok = upload((void**)&p->d_shdr, vec(p->h_shdr), p->h_shdr.size() * sizeof(SubHdr)) &&
             upload((void**)&p->d_smer, vec(p->h_smer), p->h_smer.size() * sizeof(SubMerge));
    if (!ok) {
        free_plan(p.get());
        return TDE_ENOMEM;
    }
    while (g_plan_lru.size() >= kMaxPlans) evict_plan(std::prev(g_plan_lru.end()));
    *out = p.get();
    g_plan_lru.push_front(PlanEntry{key, std::move(p)});
    g_plans.emplace(std::move(key), g_plan_lru.begin());
    return TDE_OK;
}

int resolve_opts(const tde_opts* opts, int* leaf, int* cols, int* wmin = nullptr, bool* dc = nullptr,
                 int* cap = nullptr, int* gmax = nullptr, int* wblocks = nullptr, int* ffew = nullptr) {
    int L = kDefaultLeaf, C = kDefaultSweepCols, W = kWideMin, S = kSecMaxIter, Gm = 0, Wb = 0, Ff = 0;
    if (opts) {
        if (opts->flags & ~(TDE_FLAG_NO_GRAPH | TDE_FLAG_LEAF_DC)) return TDE_EINVAL;
        if (opts->leaf != 0) L = opts->leaf;
        if (opts->sweep_cols != 0) C = opts->sweep_cols;
        if (opts->wide_min != 0) W = opts->wide_min;
        if (opts->max_sweeps != 0) S = opts->max_sweeps;
        Gm = opts->group_max;
        Wb = opts->wide_blocks;
        Ff = opts->fuse_few;
        for (int r : opts->reserved)
            if (r != 0) return TDE_EINVAL;
    }
    if (Gm != 0 && Gm != 4 && Gm != 8 && Gm != 16) return TDE_EINVAL;
    if (Wb < 0 || Wb > (1 << 20)) return TDE_EINVAL;
    if (Ff != 0 && (Ff < 2 || Ff > kFuseMaxRoots)) return TDE_EINVAL;
    if (gmax) *gmax = Gm;
    if (wblocks) *wblocks = Wb;
    if (ffew) *ffew = Ff;
    if (L < 1 || L > kLeafMax) return TDE_EINVAL;
    if (C < 1 || C > (1 << 20)) return TDE_EINVAL;
    if (W < 2) return TDE_EINVAL;
    if (S < 1 || S > kSecMaxIter) return TDE_EINVAL;
    if (cap) *cap = S;
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
    int leaf, cols, wmin, cap, gmax, wblocks, ffew;
    bool dc;
    if (resolve_opts(opts, &leaf, &cols, &wmin, &dc, &cap, &gmax, &wblocks, &ffew) != TDE_OK) return TDE_EINVAL;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return TDE_EDEVICE;
    return make_plan(device, leaf, cols, wmin, dc, gmax, wblocks, ffew, offs, plan);
}

bool needs_e(const std::vector<long long>& offs) {
    for (size_t b = 0; b + 1 < offs.size(); ++b)
        if (offs[b + 1] - offs[b] > 1) return true;
    return false;
}

int solve(const double* d, const double* e, const std::vector<long long>& offs, double* lambda, void* ws,
          size_t ws_bytes, void* stream, const tde_opts* opts, void* ckpt = nullptr, size_t ckpt_bytes = 0,
          double* qfirst = nullptr, double* qlast = nullptr) {
    int leaf, cols, wmin, cap;
    bool dc;
    if (resolve_opts(opts, &leaf, &cols, &wmin, &dc, &cap) != TDE_OK) return TDE_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
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
    w.sec_cap = cap;
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
    int leaf, cols, wmin, cap;
    bool dc;
    if (resolve_opts(opts, &leaf, &cols, &wmin, &dc, &cap) != TDE_OK) return TDE_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
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
    w.sec_cap = cap;
    Grad gr{};
    grad_layout(ntot, plan->nmerges, (char*)ws + fw, &gr);
    Ckpt ck{};
    ckpt_layout(ntot, (int)plan->levels.size(), (char*)const_cast<void*>(ckpt), &ck);
    Bufs bufs{d, e, gin, ckpt, gd, ge, ws, nullptr};
    return run_pass(*plan, PASS_BACKWARD, bufs, opts, stream,
                    [&](void* s) { return enqueue_backward(*plan, w, gr, ck, d, e, gin, gd, ge, s); });
}

// Requested rows (Algorithm 1 with an arbitrary row list sigma): the
// workspace beyond the forward's holds a forward checkpoint, the current
// nodes' vectors of the two rows a pass carries, the unsigned top rows 0 and
// n-1, a discarded eigenvalue output and the first-occurrence map.
struct SelLayout {
    size_t fw, total;
    Ckpt ck;
    double *xa, *xb, *q0, *q1, *xout;
    int* first;
};

size_t selrows_layout(long long n, long long m, int levels, char* base, SelLayout* L) {
    SelLayout t{};
    t.fw = workspace_layout(n, 1, n, nullptr, nullptr);
    size_t off = t.fw;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const long long nn = n > 0 ? n : 1;
    char* ckb = take(ckpt_layout(n, levels, nullptr, nullptr));
    ckpt_layout(n, levels, ckb, &t.ck);
    t.xa = (double*)take(8 * nn);
    t.xb = (double*)take(8 * nn);
    t.q0 = (double*)take(8 * nn);
    t.q1 = (double*)take(8 * nn);
    t.xout = (double*)take(8 * nn);
    t.first = (int*)take(4 * (m > 0 ? m : 1));
    t.total = off;
    if (L) *L = t;
    return off;
}

int selrows(const double* d, const double* e, long long n, const int64_t* rows, long long m, double* lambda,
            double* Q, void* ws, size_t ws_bytes, void* stream, const tde_opts* opts) {
    int leaf, cols, wmin, cap;
    bool dc;
    if (resolve_opts(opts, &leaf, &cols, &wmin, &dc, &cap) != TDE_OK) return TDE_EINVAL;
    if (n < 0 || n > (long long)0x3fffffff || m < 0 || m > (long long)0x3fffffff) return TDE_EINVAL;
    if (n == 0) return m == 0 ? TDE_OK : TDE_EINVAL;
    if (!d || !lambda || !ws || (n > 1 && !e) || (m > 0 && (!rows || !Q))) return TDE_EINVAL;
    for (long long i = 0; i < m; ++i)
        if (rows[i] < 0 || rows[i] >= n) return TDE_EINVAL;
    // leaves by QL (the passes rely on the leaf recurrence tracking any row)
    tde_opts o{};
    if (opts) o = *opts;
    o.flags &= ~TDE_FLAG_LEAF_DC;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    const std::vector<long long> offs{0, n};
    Plan* plan = nullptr;
    int rc = get_plan(&o, offs, &plan);
    if (rc != TDE_OK) return rc;
    SelLayout sl{};
    const int H = tree_levels(leaf, offs);
    if ((int)plan->levels.size() > H || ws_bytes < selrows_layout(n, m, H, nullptr, nullptr)) return TDE_EINVAL;
    selrows_layout(n, m, H, (char*)ws, &sl);
    // distinct rows, ascending, and the first request of each
    std::vector<int> first((size_t)(m > 0 ? m : 1));
    std::map<long long, int> slot;
    for (long long i = 0; i < m; ++i) {
        auto it = slot.find(rows[i]);
        if (it == slot.end()) it = slot.emplace(rows[i], (int)i).first;
        first[(size_t)i] = it->second;
    }
    std::vector<std::pair<long long, int>> uniq(slot.begin(), slot.end());
    Work w{};
    workspace_layout(n, 1, n, (char*)ws, &w);
    w.sec_cap = cap;
    // pass 0: eigenvalues, checkpoint, unsigned top rows 0 and n-1
    w.rows_out = 1;
    w.rows_raw = 1;
    w.qfirst = sl.q0;
    w.qlast = sl.q1;
    if (enqueue_solve(*plan, w, d, e, lambda, stream, &sl.ck) != 0) return TDE_EDEVICE;
    // one pass per two distinct rows
    for (size_t u = 0; u < uniq.size(); u += 2) {
        Work wx = w;
        wx.qfirst = wx.qlast = nullptr;
        wx.rows_raw = 0;
        wx.xmode = 1;
        wx.xa = sl.xa;
        wx.xb = sl.xb;
        wx.xa_row = uniq[u].first;
        wx.xq_a = Q + (size_t)uniq[u].second * (size_t)n;
        if (u + 1 < uniq.size()) {
            wx.xb_row = uniq[u + 1].first;
            wx.xq_b = Q + (size_t)uniq[u + 1].second * (size_t)n;
        } else {
            wx.xb_row = -1;
            wx.xq_b = nullptr;
        }
        if (enqueue_solve(*plan, wx, d, e, sl.xout, stream, nullptr, &sl.ck) != 0) return TDE_EDEVICE;
    }
    if (m > 0) {
        if (hipMemcpyAsync(sl.first, first.data(), sizeof(int) * (size_t)m, hipMemcpyHostToDevice,
                           (hipStream_t)stream) != hipSuccess)
            return TDE_EDEVICE;
        if (enqueue_selrows_fix(Q, m, n, sl.first, sl.q0, sl.q1, stream) != 0) return TDE_EDEVICE;
        // the host map must outlive the copy: wait for it (pageable memory)
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return TDE_EDEVICE;
    }
    return TDE_OK;
}

// Driver pre-pass: pairwise merge schedule of the blocks of every problem
// (balanced over the blocks, levelled by height), cached per split.
// Bounded, least recently used first out; an evicted schedule's table is
// freed after the device has finished with it.
struct RunMerges {
    std::vector<std::pair<int, int>> levels;  // (first record, count) per pass
    MergeRec* d_recs = nullptr;
    int device = 0;
};
using RunKey = std::tuple<int, std::vector<long long>, std::vector<long long>>;
constexpr size_t kMaxRunSchedules = 32;
struct RunEntry {
    RunKey key;
    RunMerges rm;
};
std::list<RunEntry> g_run_lru;  // front = most recently used
std::map<RunKey, std::list<RunEntry>::iterator> g_runs;

void free_runs(RunMerges* rm) {
    if (!rm->d_recs) return;
    DeviceScope ds(rm->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(rm->d_recs);
    rm->d_recs = nullptr;
}

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
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    RunKey key{device, offs, nb};
    auto it = g_runs.find(key);
    if (it != g_runs.end()) {
        g_run_lru.splice(g_run_lru.begin(), g_run_lru, it->second);
        *out = &it->second->rm;
        return TDE_OK;
    }
    while (g_run_lru.size() >= kMaxRunSchedules) {
        auto last = std::prev(g_run_lru.end());
        free_runs(&last->rm);
        g_runs.erase(last->key);
        g_run_lru.erase(last);
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
    rm.device = device;
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
    g_run_lru.push_front(RunEntry{key, std::move(rm)});
    g_runs.emplace(std::move(key), g_run_lru.begin());
    *out = &g_run_lru.front().rm;
    return TDE_OK;
}

int solve_split(const double* d, const double* e, const std::vector<long long>& offs, double* lambda, void* ws,
                size_t ws_bytes, void* stream, const tde_opts* opts, int64_t* nblocks) {
    int leaf, cols;
    if (resolve_opts(opts, &leaf, &cols) != TDE_OK) return TDE_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
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

int tde_version(void) { return 201; }

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

size_t tde_selrows_workspace_bytes(int64_t n, int64_t m, const tde_opts* opts) {
    int leaf, cols;
    if (n < 0 || m < 0 || tde::resolve_opts(opts, &leaf, &cols) != TDE_OK) return 0;
    const std::vector<long long> offs{0, (long long)n};
    return tde::selrows_layout(n, m, tde::tree_levels(leaf, offs), nullptr, nullptr);
}

int tde_eigvals_selrows(const double* d, const double* e, int64_t n, const int64_t* rows, int64_t m,
                        double* lambda, double* Q, void* ws, size_t ws_bytes, void* hip_stream,
                        const tde_opts* opts) {
    return tde::selrows(d, e, (long long)n, rows, (long long)m, lambda, Q, ws, ws_bytes, hip_stream, opts);
}

size_t tde_dense_workspace_bytes(int64_t n, const tde_opts* opts) {
    int leaf, cols;
    if (n < 0 || n > (int64_t)0x3fffffff || tde::resolve_opts(opts, &leaf, &cols) != TDE_OK) return 0;
    return tde::dense_layout(n, nullptr, nullptr) + tde::workspace_layout(n, 1, n, nullptr, nullptr);
}

int tde_dense_eigvals(double* A, int64_t n, int64_t lda, double* lambda, double* d_out, double* e_out, void* ws,
                      size_t ws_bytes, void* hip_stream, const tde_opts* opts) {
    int leaf, cols;
    if (n < 0 || n > (int64_t)0x3fffffff || tde::resolve_opts(opts, &leaf, &cols) != TDE_OK) return TDE_EINVAL;
    if (n == 0) return TDE_OK;
    if (!A || !lambda || !ws || lda < n) return TDE_EINVAL;
    // the solver's workspace first (its status word is where tde_get_status
    // looks), the reduction's scratch after it
    const size_t sb = tde::workspace_layout(n, 1, n, nullptr, nullptr);
    if (ws_bytes < sb + tde::dense_layout(n, nullptr, nullptr)) return TDE_EINVAL;
    tde::DenseWork dw{};
    tde::dense_layout(n, (char*)ws + sb, &dw);
    const std::vector<long long> offs{0, (long long)n};
    {
        // the reduction's launches (three per column) are captured once per
        // (size, buffers) into a graph, like the solve's
        std::lock_guard<std::recursive_mutex> lk(tde::g_mu);
        tde::Plan* plan = nullptr;
        const int rc = tde::get_plan(opts, offs, &plan);
        if (rc != TDE_OK) return rc;
        const tde::Bufs bufs{A, ws, (const void*)(intptr_t)lda, nullptr, nullptr, nullptr, nullptr, nullptr};
        const int rr = tde::run_pass(*plan, tde::PASS_DENSE, bufs, opts, hip_stream, [&](void* s) {
            return tde::enqueue_dense_reduce(A, lda, (int)n, dw, s);
        });
        if (rr != TDE_OK) return rr;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (d_out && hipMemcpyAsync(d_out, dw.d, 8 * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TDE_EDEVICE;
    if (e_out && n > 1 && hipMemcpyAsync(e_out, dw.e, 8 * (size_t)(n - 1), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TDE_EDEVICE;
    return tde::solve(dw.d, dw.e, offs, lambda, ws, sb, hip_stream, opts);
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
    std::lock_guard<std::recursive_mutex> lk(tde::g_mu);
    while (!tde::g_plan_lru.empty()) tde::evict_plan(std::prev(tde::g_plan_lru.end()));
    tde::drop_graphs_if([](const tde::GraphEntry&) { return true; });
    for (auto& r : tde::g_run_lru) tde::free_runs(&r.rm);
    tde::g_run_lru.clear();
    tde::g_runs.clear();
}

int tde_cache_sizes(int64_t* out, int n) {
    if (!out || n < 0) return TDE_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(tde::g_mu);
    const int64_t v[3] = {(int64_t)tde::g_plan_lru.size(), (int64_t)tde::g_graph_lru.size(),
                          (int64_t)tde::g_run_lru.size()};
    for (int k = 0; k < n && k < 3; ++k) out[k] = v[k];
    return TDE_OK;
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
