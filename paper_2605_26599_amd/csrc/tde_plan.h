// Host-side plan of a (batched) BR D&C solve: the static merge tree of every
// problem, levelled by height so that all merges of one height run together.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "tde_internal.h"

namespace tde {

struct LevelInfo {
    int mstart;   // first merge of this level in the flat merge table
    int M;        // merges in this level
    long long N;  // packed columns in this level (sum of merge sizes)
    int smax;     // largest merge (columns) in this level
    int bstart;   // first entry of this level's per-block merge table
    int wpstart;  // levels of merges of at most kLeafMax columns: first entry of the
                  // in-wave pack table (first merge of every pack, then M) in h_blkm
    int nwp;      // packs of such a level (0: none)
    int all_root; // 1 when every merge of the level is a problem's top merge
};

struct Plan {
    int device = 0;
    long long ntot = 0;
    int B = 0;
    int leaf = 32;
    int sweep_cols = 8;  // target poles per lane in the root-parallel sweeps
    int wide_min = kWideMin;  // merges with at least this many active roots use the wide secular sweep
    bool leaf_dc = false;     // forward passes solve the leaves by divide and conquer inside one wave
    int group_max = 0;        // lanes per root in the fused small merges (4, 8, 16); 0 = by level
    int wide_blocks = 0;      // most workgroups of a wide root launch; 0 = default (4096)
    int fuse_few = 0;         // fused limit on levels of few merges (active roots); 0 = kFuseMax
    int nleaves = 0;
    int leafmax = 1;     // largest leaf size in the plan
    int maxM = 1;        // most merges in one level
    long long maxN = 1;  // most packed columns in one level
    std::vector<long long> offs;  // host copy of the problem offsets [B+1]
    std::vector<LevelInfo> levels;
    // host tables (plan_host), uploaded to the device tables below
    std::vector<MergeRec> h_merges;  // every merge, level after level
    std::vector<int> h_blkm;         // per level, per block of kWG packed columns: first merge touched;
                                     // then the level's in-wave pack table, if any
    std::vector<LeafRec> h_leaves;
    std::vector<SubHdr> h_shdr;      // in-wave merge trees by leaf size (leaf_dc only)
    std::vector<SubMerge> h_smer;
    // device tables owned by the plan
    int nmerges = 0;           // merges over all levels
    MergeRec* d_merges = nullptr;
    int* d_blkm = nullptr;     // per level, per block of kWG packed columns: first merge touched
    LeafRec* d_leaves = nullptr;
    long long* d_offs = nullptr;
    SubHdr* d_shdr = nullptr;      // [kLeafMax+1] in-wave merge trees by leaf size (leaf_dc)
    SubMerge* d_smer = nullptr;
};

// Host tables of a plan from p->offs, p->leaf and p->leaf_dc (levels, merges,
// leaves, block-to-merge map, in-wave trees).  0, or -1 when the tree has more
// levels than the per-level counters hold.
int plan_host(Plan* p);
void sub_trees(std::vector<SubHdr>* hdr, std::vector<SubMerge>* mer);

// Workspace layout for n packed columns, B problems and maxM merges per level.
// With base == nullptr only the size is computed.
size_t workspace_layout(long long n, long long B, long long maxM, char* base, Work* w);

// Optional per-kernel timing (HIP events around every launch, per kind).
void timing_enable(bool on);
bool timing_enabled();
// Launches enqueued by the calling thread are (not) timed, whatever
// timing_enable says (timing creates events, which the allocation-free entry
// point must not do).
void timing_suppress(bool on);
int timing_read(double* ms, long long* count, int nkinds);

// Reverse-pass scratch (n columns, nmerges merges) and forward checkpoint
// (n columns, `levels` tree levels).  With base == nullptr only the size.
size_t grad_layout(long long n, long long nmerges, char* base, Grad* g);
size_t ckpt_layout(long long n, int levels, char* base, Ckpt* c);

// Enqueue one full solve (scale, leaves, every level) on stream; with ck, also
// record the checkpoint the reverse pass reads.
int enqueue_solve(const Plan& p, const Work& w, const double* d, const double* e, double* out, void* stream,
                  const Ckpt* ck = nullptr, const Ckpt* xsrc = nullptr);
// With xsrc (a requested-rows pass, w.xmode = 1): every level reads its node
// spectra and boundary rows from the checkpoint xsrc of a forward solve of the
// same inputs and plan instead of the workspace.

// Requested rows: sign the columns of Q [m][n] by the unsigned top rows q0, q1
// (first entry >= 0) and copy repeated rows from their first occurrence
// first[i] (device).
int enqueue_selrows_fix(double* Q, long long m, long long n, const int* first, const double* q0,
                        const double* q1, void* stream);

// Driver pre-pass: negligible-coupling flags (flags[i] = 1: a block starts at
// column i), and one pass of pairwise merges of ascending runs (src -> dst).
int enqueue_split_flags(const double* d, const double* e, long long n, int* flags, void* stream);
int enqueue_merge_runs(const MergeRec* recs, int M, const double* src, double* dst, long long n, void* stream);

// Enqueue the reverse pass: gd, ge = d(sum_k gin_k lambda_k)/d(d, e) from the
// checkpoint of a forward solve of the same (d, e) under the same plan.
int enqueue_backward(const Plan& p, const Work& w, const Grad& gr, const Ckpt& ck, const double* d,
                     const double* e, const double* gin, double* gd, double* ge, void* stream);

}  // namespace tde
