// Allocation-free variant of tde_eigvals for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The workspace and the plan's merge-tree tables live in one file-scope
// device array, `scratch`, of kScratchBytes; each GPU the library runs on
// holds its own copy until the process ends.  The host never uses the array's
// name as an address (in host code it names a host-side stand-in): the
// device address is looked up once per device with hipGetSymbolAddress and
// kept.  Each call uploads its tables into the array with an asynchronous
// copy on the caller's stream and enqueues the kernels one by one on that
// stream (no graph: instantiating one allocates), so consecutive calls on one
// stream are ordered; calls that overlap on one GPU (two streams, or two
// threads) share the array and race.
#include <hip/hip_runtime.h>

#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/tde.h"
#include "tde_plan.h"

namespace tde {
namespace {

constexpr long long kNoAllocMaxN = 65536;       // largest problem the scratch array holds
constexpr size_t kScratchBytes = 24ull << 20;   // workspace (~284 B per column) + tree tables

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_na_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of that device's scratch

// Host-only plans (no device tables of their own), least recently used out.
using NaKey = std::tuple<long long, int, int, int, bool, int, int, int>;
constexpr size_t kMaxNaPlans = 16;
struct NaEntry {
    NaKey key;
    std::unique_ptr<Plan> plan;
};
std::list<NaEntry> g_na_lru;
std::map<NaKey, std::list<NaEntry>::iterator> g_na_plans;

// Device address of `scratch` on the current device (looked up once per device).
int scratch_for(int device, char** out) {
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return TDE_OK;
    }
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TDE_EDEVICE;
    g_scratch_ptr[device] = (char*)ptr;
    *out = (char*)ptr;
    return TDE_OK;
}

const Plan* host_plan(long long n, int leaf, int cols, int wmin, bool dc, int gmax, int wblocks, int ffew) {
    NaKey key{n, leaf, cols, wmin, dc, gmax, wblocks, ffew};
    auto it = g_na_plans.find(key);
    if (it != g_na_plans.end()) {
        g_na_lru.splice(g_na_lru.begin(), g_na_lru, it->second);
        return it->second->plan.get();
    }
    auto p = std::make_unique<Plan>();
    p->leaf = leaf;
    p->sweep_cols = cols;
    p->wide_min = wmin;
    p->leaf_dc = dc;
    p->group_max = gmax;
    p->wide_blocks = wblocks;
    p->fuse_few = ffew;
    p->offs = {0, n};
    if (plan_host(p.get()) != 0) return nullptr;
    while (g_na_lru.size() >= kMaxNaPlans) {
        // the staged host-to-device copies of an evicted plan read its host
        // tables before hipMemcpyAsync returned (pageable source memory)
        g_na_plans.erase(g_na_lru.back().key);
        g_na_lru.pop_back();
    }
    g_na_lru.push_front(NaEntry{key, std::move(p)});
    g_na_plans.emplace(key, g_na_lru.begin());
    return g_na_lru.front().plan.get();
}

int eigvals_noalloc(const double* d, const double* e, long long n, double* lambda, int* status, void* stream,
                    const tde_opts* opts) {
    int L = kDefaultLeaf, C = kDefaultSweepCols, W = kWideMin, S = kSecMaxIter, Gm = 0, Wb = 0, Ff = 0;
    bool dc = false;
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
        dc = (opts->flags & TDE_FLAG_LEAF_DC) != 0;
    }
    if (L < 1 || L > kLeafMax || C < 1 || C > (1 << 20) || W < 2 || S < 1 || S > kSecMaxIter) return TDE_EINVAL;
    if (Gm != 0 && Gm != 4 && Gm != 8 && Gm != 16) return TDE_EINVAL;
    if (Wb < 0 || Wb > (1 << 20)) return TDE_EINVAL;
    if (Ff != 0 && (Ff < 2 || Ff > kFuseMaxRoots)) return TDE_EINVAL;
    if (n < 0 || n > kNoAllocMaxN) return TDE_EINVAL;
    if (n == 0) return TDE_OK;
    if (!d || !lambda || (n > 1 && !e)) return TDE_EINVAL;

    std::lock_guard<std::mutex> lk(g_na_mu);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return TDE_EDEVICE;
    char* base = nullptr;
    int rc = scratch_for(device, &base);
    if (rc != TDE_OK) return rc;
    const Plan* hp = host_plan(n, L, C, W, dc, Gm, Wb, Ff);
    if (!hp) return TDE_EINVAL;

    // carve the scratch: tree tables first, then the workspace
    Plan p = *hp;  // host copy whose device-table pointers point into scratch
    size_t off = 0;
    bool fits = true;
    auto take = [&](size_t bytes) -> char* {
        char* q = base + off;
        off += (bytes + 255) & ~(size_t)255;
        if (off > kScratchBytes) fits = false;
        return q;
    };
    p.device = device;
    p.d_merges = (MergeRec*)take(p.h_merges.size() * sizeof(MergeRec));
    p.d_leaves = (LeafRec*)take(p.h_leaves.size() * sizeof(LeafRec));
    p.d_offs = (long long*)take(p.offs.size() * sizeof(long long));
    p.d_blkm = (int*)take(p.h_blkm.size() * sizeof(int));
    p.d_shdr = dc ? (SubHdr*)take(p.h_shdr.size() * sizeof(SubHdr)) : nullptr;
    p.d_smer = dc ? (SubMerge*)take(p.h_smer.size() * sizeof(SubMerge)) : nullptr;
    char* wsbase = take(0);
    const size_t wsb = workspace_layout(n, 1, n, nullptr, nullptr);
    if (!fits || off + wsb > kScratchBytes) return TDE_EINVAL;
    Work w{};
    workspace_layout(n, 1, n, wsbase, &w);
    w.sec_cap = S;

    hipStream_t s = (hipStream_t)stream;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    if (!up(p.d_merges, hp->h_merges.data(), hp->h_merges.size() * sizeof(MergeRec)) ||
        !up(p.d_leaves, hp->h_leaves.data(), hp->h_leaves.size() * sizeof(LeafRec)) ||
        !up(p.d_offs, hp->offs.data(), hp->offs.size() * sizeof(long long)) ||
        !up(p.d_blkm, hp->h_blkm.data(), hp->h_blkm.size() * sizeof(int)) ||
        (dc && !up(p.d_shdr, hp->h_shdr.data(), hp->h_shdr.size() * sizeof(SubHdr))) ||
        (dc && !up(p.d_smer, hp->h_smer.data(), hp->h_smer.size() * sizeof(SubMerge))))
        return TDE_EDEVICE;

    timing_suppress(true);
    rc = enqueue_solve(p, w, d, e, lambda, stream);
    timing_suppress(false);
    if (rc != 0) return TDE_EDEVICE;
    if (status && hipMemcpyAsync(status, w.status, sizeof(int), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TDE_EDEVICE;
    return TDE_OK;
}

}  // namespace
}  // namespace tde

extern "C" int tde_eigvals_noalloc(const double* d, const double* e, int64_t n, double* lambda, int* status,
                                   void* hip_stream, const tde_opts* opts) {
    return tde::eigvals_noalloc(d, e, (long long)n, lambda, status, hip_stream, opts);
}
