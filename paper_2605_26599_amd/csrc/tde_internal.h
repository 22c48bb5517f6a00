// Internal data layout shared by the host plan and the gfx950 kernels of the
// boundary-row divide-and-conquer (BR D&C) tridiagonal eigenvalue solver.
#pragma once
#include <stdint.h>

namespace tde {

// One rank-one merge of the D&C tree (paper Section 3.1, merge problem).
// The parent node covers global elements [off, off + nL + nR); its left child
// is [off, off + nL) and its right child [off + nL, off + nL + nR).  The tear
// coupling is e[off + nL - 1].  Merges of one tree level are packed back to
// back: this merge's scratch rows start at packed position pk.
struct MergeRec {
    long long off;
    long long pk;
    int nL;
    int nR;
    int prob;   // problem index within the batch
    int flags;  // MF_ROOT: top merge of its problem (eigenvalues only, no rows)
};
enum { MF_ROOT = 1 };

// One leaf of the D&C tree: global elements [off, off + size) of problem prob.
struct LeafRec {
    long long off;
    int size;
    int prob;
    int flags;  // LF_TEAR_LEFT / LF_TEAR_RIGHT: a tear coupling sits on that side;
                // LF_WHOLE: the leaf is the whole problem (write the output directly)
    int pad;
};
enum { LF_TEAR_LEFT = 1, LF_TEAR_RIGHT = 2, LF_WHOLE = 4 };

// Merge tree of a leaf solved by divide and conquer inside one wave (the
// leaf's own balanced halving down to single columns, levelled by height, the
// same shape the global tree has below that node).  Offsets are local to the
// leaf.  Per leaf size l: SubHdr[l] gives the first SubMerge of the size and,
// for local level h < H, the merges [lv[h], lv[h+1]) of that level.
struct SubMerge {
    unsigned char off, nL, nR, pk;
};
struct SubHdr {
    int mbase;
    int H;
    unsigned char lv[8];
};

// Device status bits (OR-ed into the status word at the start of the workspace).
enum {
    ST_NONFINITE = 1,  // NaN or Inf in d or e
    ST_LEAF_NOCONV = 2,
    ST_SEC_NOCONV = 4,
};

// Work counters (Work::counters), reset at the start of every solve.
enum {
    CNT_SEC_TERMS = 0,   // pole-term evaluations in secular sweeps
    CNT_LOW_PAIRS = 1,   // (pole, root) pairs in the Loewner products
    CNT_ROW_PAIRS = 2,   // (root, pole) pairs in the boundary-row dot products
    CNT_ROOTS = 3,       // secular roots solved
    CNT_SWEEPS = 4,      // secular sweeps (summed over roots)
    CNT_LEAF_COLS = 5,   // columns solved by the QL leaf kernel
    CNT_LEAF_ROT = 6,    // plane rotations applied by the QL leaf kernel
    CNT_MERGE_COLS = 7,  // columns passed through merges (summed over levels)
    // the same work done inside leaves solved by divide and conquer in one wave
    CNT_DC_TERMS = 8,      // pole-term evaluations in secular sweeps
    CNT_DC_LOW_PAIRS = 9,  // (pole, root) pairs in the Loewner products
    CNT_DC_ROW_PAIRS = 10, // (root, pole) pairs in the boundary-row dot products
    CNT_DC_ROOTS = 11,     // secular roots solved
    // the part of [0..3] done by the fused kernel of merges with few active roots
    CNT_SM_TERMS = 12,
    CNT_SM_LOW_PAIRS = 13,
    CNT_SM_ROW_PAIRS = 14,
    CNT_SM_ROOTS = 15,
    // the same for the whole-merge workgroups of small levels (k_level_block)
    CNT_LB_TERMS = 16,
    CNT_LB_LOW_PAIRS = 17,
    CNT_LB_ROW_PAIRS = 18,
    CNT_LB_ROOTS = 19,
    CNT_N = 20
};
// Each counter is spread over kCntSlots words (a launch's waves add into
// different slots, so their atomics do not queue on one address); readers sum
// the slots.  The slots sit at byte kCntOffset of the workspace.
constexpr int kCntSlots = 64;
constexpr int kCntOffset = 256;

// Launch kinds for the optional per-kernel timing.
enum {
    KIND_SETUP = 0, KIND_LEAF, KIND_MERGE, KIND_DEFLATE, KIND_SECULAR, KIND_LOWNER, KIND_ROWS, KIND_ASSEMBLE,
    KIND_BACKWARD, KIND_SMALL, KIND_LEVEL, KIND_N
};

constexpr int kWG = 256;         // threads per workgroup for element-parallel kernels
constexpr int kLeafMax = 64;     // largest leaf the QL leaf kernel accepts
constexpr int kFuseMaxRoots = 512;  // most active roots of a merge one fused workgroup solves
constexpr int kDefaultLeaf = 8;  // leaf size when the caller does not choose one
constexpr int kDefaultSweepCols = 8;  // poles per lane per sweep when the caller does not choose
constexpr int kSecMaxIter = 96;  // secular iteration cap
constexpr int kWideMin = 1024;   // merges with at least this many active roots use the wide secular sweep
constexpr int kWideWaves = 4;    // pole segments (waves) per workgroup of the wide secular sweep
constexpr int kMaxLevels = 40;   // tree levels the per-level block counters can hold
constexpr int kSelfScanMax = 2048;  // up to this many blocks per level, blocks sum their own count prefixes

// Pointers into the caller's workspace for one solve.
struct Work {
    int* status;               // [1]   device status bits
    unsigned long long* counters;  // [CNT_N][kCntSlots] algorithmic work of the last solve (CNT_*)
    unsigned long long* pmax;  // [B]   bits of max |d|,|e| per problem
    double* lam;               // [n]   node spectra (ascending per node)
    double* blo;               // [n]   node first eigenvector row
    double* bhi;               // [n]   node last eigenvector row
    double* D;                 // [n]   merged, sorted poles (packed per level)
    double* Z;                 // [n]   secular vector z~ in pole order
    double* RL;                // [n]   parent-first-row entries per column
    double* RH;                // [n]   parent-last-row entries per column
    int* src;                  // [n]   local child column that landed at each merged position
    double* D2;                // [n]   candidates after close-pole rotations
    double* Z2;                // [n]
    double* RL2;               // [n]
    double* RH2;               // [n]
    int* st;                   // [n]   column state: 0 negligible z, 1 active, 2 rotated away
    int* scan;                 // [n + n/2 + 2] exclusive prefix counts of active columns (level-wide, or per merge)
    int* scanC;                // [n + n/2 + 2] the same for candidate (non-negligible) columns
    int* scanR;                // [n + n/2 + 2] the same for rotated-away columns
    int* bsum;                 // [nb+1] per-block counts
    int* bsumR;                // [nb+1] per-block counts of rotated-away columns (this level's slice of bcnt)
    int* bsumA;                // [nb+1] per-block counts of active columns (raw; this level's slice of bcnt)
    int* bcnt;                 // [kMaxLevels][2][nb+2] per-level block counts, zeroed once per pass
    int* bsumAs;               // [nb+1] exclusive scan of bsumA
    int* bsumRs;               // [nb+1] exclusive scan of bsumR
    unsigned* ticket;          // [1]   last-workgroup ticket (self-resetting)
    int* nnpos;                // [n]   packed positions of non-negligible columns
    int* cf;                   // [n]   close-pair flag of non-negligible column g and g+1
    double* Da;                // [n]   active poles
    double* Za;                // [n]   active z
    double* Wa;                // [n]   active z^2 (the weights the wide secular sweep reads)
    double* RLa;               // [n]
    double* RHa;               // [n]
    int* amerge;               // [n]   merge index (within the level) of active column g
    int* witems;               // [maxM+1] exclusive scan of 64-root blocks per wide merge
    int* apos;                 // [n]   packed position of active column g
    int* rpos;                 // [n]   packed position of rotated-away column gr
    int* dpos;                 // [n]   packed position of negligible-z column q
    int* org;                  // [n]   root origin (local active index)
    double* tau;               // [n]   root offset from its origin pole
    double* rootval;           // [n]   the root itself, D_org + tau (what the assembly sorts by)
    double* dorg;              // [n]   D_org of the roots of wide merges (forward; read by their Loewner step)
    double* zhat;              // [n]   recomputed (Loewner) secular vector
    double* PBL;               // [n]   parent first-row entries of active columns
    double* PBH;               // [n]   parent last-row entries of active columns
    double* Dd;                // [n]   negligible-z columns: eigenvalue D_j (ascending per merge)
    double* RLd;               // [n]
    double* RHd;               // [n]
    double* Dr;                // [n]   rotated-away columns: eigenvalue (ascending per merge)
    double* RLr;               // [n]
    double* RHr;               // [n]
    double* qfirst;            // [n] or null: first eigenvector row of each output eigenvalue (rows mode)
    double* qlast;             // [n] or null: last eigenvector row of each output eigenvalue (rows mode)
    int rows_out;              // 1: the top merges also propagate rows (qfirst / qlast requested)
    int sec_cap;               // secular iterations allowed per root before ST_SEC_NOCONV (kSecMaxIter)
    int rows_raw;              // rows mode: store the top rows as computed (no sign normalisation)
    // Requested-rows pass (xmode = 1): the two row channels carry rows xa_row and
    // xb_row of every node that contains them (global indices, -1 = none) instead
    // of the parent's first and last rows; z still comes from the node boundary
    // rows (lam, blo, bhi then point at a forward checkpoint's level slot, read
    // only).  xa / xb hold those rows of the current nodes (global positions, in
    // place across levels); the top merge writes them to xq_a / xq_b (length n).
    int xmode;
    long long xa_row, xb_row;
    double* xa;
    double* xb;
    double* xq_a;
    double* xq_b;
};

// Forward checkpoint for the reverse pass: per level h (slot stride n), the
// node spectra and rows that level's merges read (global positions) and the
// level's secular roots as (org, tau) by active index.  Everything else of a
// level (merged order, deflation, Loewner z) is recomputed from these.
struct Ckpt {
    double* lam;   // [H][n]
    double* blo;   // [H][n]
    double* bhi;   // [H][n]
    double* tau;   // [H][n]
    int* org;      // [H][n]
    long long n;   // slot stride
};

// One column's state in a close-pole run: pole, z, parent first/last-row entries.
struct RunState {
    double D, Z, L, H;
};

// Reverse-pass scratch: adjoints of one level's quantities (packed like the
// forward's level arrays) and of the node spectra/rows (global positions).
struct Grad {
    double* glam;  // [n] node adjoints: dL/dlambda of each node column (in place across levels)
    double* gblo;  // [n] dL/dblo
    double* gbhi;  // [n] dL/dbhi
    double* gD;    // [n] adjoints of the merged (pre-rotation) columns, packed per level
    double* gZ;
    double* gRL;
    double* gRH;
    double* gD2;   // [n] adjoints of the post-rotation columns, packed per level
    double* gZ2;
    double* gRL2;
    double* gRH2;
    double* glr;   // [n] per active root: dL/dlambda_k, dL/dblo_k, dL/dbhi_k
    double* gbr;
    double* ghr;
    double* coef;  // [10 n] per active root: 10 coefficient planes of stride n (see bwd_root_coeffs)
    RunState* chain;  // [n] run states by candidate index
    RunState* cdef;   // [n] rotated-away columns of a run, unsorted, by candidate index
    double* skey;     // [n] rotated-away poles by candidate index (sort keys)
    int* sidx;        // [n] sorted slot -> candidate index of the rotated-away column
    double* grho;     // [merges, flat over levels] dL/drho~
    double* gdp;      // [n] dL/dd' (torn diagonal)
};

}  // namespace tde
