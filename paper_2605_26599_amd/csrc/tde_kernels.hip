// gfx950 kernels of the boundary-row divide-and-conquer eigenvalue solver and
// the launch sequence of one solve.  All arithmetic lives in tde_device.h; the
// kernels here map threads to columns, roots or leaves, aggregate per-merge
// maxima and prefix counts, and order the steps of each tree level.
#include <hip/hip_runtime.h>

#include "tde_adjoint.h"
#include "tde_plan.h"

#include <mutex>
#include <vector>

namespace tde {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
// Start of a pass: zero the status words, the work counters, the per-problem
// maxima and the per-level block counts in one launch.
__global__ void k_setup(int* status, long long nst, unsigned long long* counters, long long ncnt,
                        unsigned long long* pmax, long long B, int* bcnt, long long nbc) {
    const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x, st = (long long)gridDim.x * blockDim.x;
    for (long long i = t0; i < nst; i += st) status[i] = 0;
    for (long long i = t0; i < ncnt; i += st) counters[i] = 0ULL;
    for (long long i = t0; i < B; i += st) pmax[i] = 0ULL;
    for (long long i = t0; i < nbc; i += st) bcnt[i] = 0;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long u = __shfl_xor(v, o, 64);
        v = (u > v) ? u : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Adds a per-lane count to work counter `which` with one atomic per wave,
// into the slot of this wave.
__device__ __forceinline__ unsigned long long* count_slot(unsigned long long* c, int which) {
    return c + which * kCntSlots + (((blockIdx.x << 2) + (threadIdx.x >> 6)) & (kCntSlots - 1));
}
__device__ __forceinline__ void count_add(unsigned long long* c, int which, unsigned long long v) {
    v = wave_sum_u64(v);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(count_slot(c, which), v);
}
// The same for a count held by one lane.
__device__ __forceinline__ void count_add1(unsigned long long* c, int which, unsigned long long v) {
    if (v) atomicAdd(count_slot(c, which), v);
}

// Non-finite input (flagged by k_maxabs, the first kernel of a pass): every
// later kernel of the pass returns at once.  Sorting NaNs is not a
// permutation, so the per-level counts could not be trusted; the output is
// undefined and the status word reports TDE_ENONFINITE.
__device__ __forceinline__ bool input_nonfinite(const Work& w) {
    // the bit is set by an earlier launch: a cached scalar read sees it
    return (*(const __attribute__((address_space(4))) int*)w.status & ST_NONFINITE) != 0;
}

// Inclusive scan over the workgroup (blockDim.x <= 1024, multiple of 64).
__device__ __forceinline__ int block_incl_scan(int v, int* wsum) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    if (wid == 0) {
        int x = (lane < nw) ? wsum[lane] : 0;
        for (int d = 1; d < 16; d <<= 1) {
            int u = __shfl_up(x, d, 64);
            if (lane >= d) x += u;
        }
        if (lane < nw) wsum[lane] = x;
    }
    __syncthreads();
    if (wid > 0) v += wsum[wid - 1];
    return v;
}

// Exclusive scans of the per-block counts in[0..nb) into out[0..nb], totals
// in out[nb]; a second array pair is scanned when in2 is given.  Each thread
// takes a run of consecutive counts (loaded together), so one workgroup scan
// covers them all.
__global__ __launch_bounds__(1024) void k_scan_blocks(const int* in, int* out, const int* in2, int* out2, int nb) {
    __shared__ int wsum[16];
    const int cs = (nb + 1023) / 1024;
    const int b0 = min(nb, (int)threadIdx.x * cs), b1 = min(nb, b0 + cs);
    int s1 = 0, s2 = 0;
#pragma unroll 4
    for (int i = b0; i < b1; ++i) {
        s1 += in[i];
        if (in2) s2 += in2[i];
    }
    const int incl = block_incl_scan(s1, wsum);
    __syncthreads();
    const int incl2 = block_incl_scan(s2, wsum);
    int r1 = incl - s1, r2 = incl2 - s2;
    for (int i = b0; i < b1; ++i) {
        out[i] = r1;
        r1 += in[i];
        if (in2) {
            out2[i] = r2;
            r2 += in2[i];
        }
    }
    if (threadIdx.x == 1023) {
        out[nb] = incl;
        if (in2) out2[nb] = incl2;
    }
}

// ---------------------------------------------------------------------------
// Validation and scale: pmax[b] = bits of max(|d|, |e|) over problem b;
// non-finite entries raise ST_NONFINITE.  A workgroup covers kMaxAbsPer * kWG
// consecutive entries (kMaxAbsPer per thread, kWG apart, so every load is
// coalesced); a thread folds its entries per problem and flushes a problem's
// running maximum when it moves to the next, and a workgroup whose threads all
// end in one problem issues a single atomic for all of them (one problem of
// 65536 entries: 64 atomics on its word instead of one per wave).
// ---------------------------------------------------------------------------
constexpr int kMaxAbsPer = 4;
__global__ __launch_bounds__(kWG) void k_maxabs(const double* __restrict__ d, const double* __restrict__ e,
                                                const long long* __restrict__ offs, int B, long long ntot,
                                                unsigned long long* pmax, int* status) {
    __shared__ unsigned long long sv[kWG / 64];
    __shared__ int sb[kWG / 64];
    const long long base = (long long)blockIdx.x * (kWG * kMaxAbsPer) + threadIdx.x;
    int bc = -1, blo = 0;
    long long bend = -1;  // end of problem blo
    unsigned long long vc = 0;
    bool fin = true;
    for (int k = 0; k < kMaxAbsPer; ++k) {
        const long long i = base + (long long)k * kWG;
        if (i >= ntot) break;
        if (i >= bend) {  // entries ascend, so problems never go back
            int lo = blo, hi = B - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (offs[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            blo = lo;
            bend = offs[lo + 1];
        }
        const int lo = blo;
        double x = fabs(d[i]);
        bool f = x <= DBL_MAX;
        if (i + 1 < bend) {
            const double y = fabs(e[i]);
            f = f && (y <= DBL_MAX);
            x = fmax(x, y);
        }
        fin = fin && f;
        if (lo != bc) {
            if (bc >= 0) atomicMax(&pmax[bc], vc);
            bc = lo;
            vc = 0;
        }
        const unsigned long long u = dbits(x);
        vc = (u > vc) ? u : vc;
    }
    if (!fin) atomicOr(status, ST_NONFINITE);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b0 = __shfl(bc, 0, 64);
    const bool wave_one = __all(bc == b0);
    if (wave_one) vc = wave_max_u64(vc);
    if (lane == 0) {
        sb[wv] = wave_one ? b0 : -2;
        sv[wv] = vc;
    }
    __syncthreads();
    bool block_one = true;
    unsigned long long vb = 0;
    for (int q = 0; q < kWG / 64; ++q) {
        block_one = block_one && (sb[q] == sb[0]);
        vb = (sv[q] > vb) ? sv[q] : vb;
    }
    if (block_one) {
        if (threadIdx.x == 0 && sb[0] >= 0) atomicMax(&pmax[sb[0]], vb);
    } else if (wave_one) {
        if (lane == 0 && b0 >= 0) atomicMax(&pmax[b0], vc);
    } else if (bc >= 0) {
        atomicMax(&pmax[bc], vc);
    }
}

// ---------------------------------------------------------------------------
// Leaves: one lane per leaf, `per` leaves per wave (lanes 0..per-1), the
// leaf's working arrays in LDS (lane-strided).  A wave's leaves run their QL
// iterations in lockstep and wait for one another's extra sweeps, so with few
// leaves fewer share a wave and more waves run side by side.
// ---------------------------------------------------------------------------
template <int LMAX>
__global__ __launch_bounds__(64) void k_leaf(const LeafRec* __restrict__ leaves, int nleaves,
                                             const double* __restrict__ d, const double* __restrict__ e,
                                             const unsigned long long* __restrict__ pmax, Work w,
                                             double* __restrict__ out, int per) {
    if (input_nonfinite(w)) return;
    __shared__ double sd[LMAX * 64], se[LMAX * 64], s0[LMAX * 64], s1[LMAX * 64];
    const int lane = threadIdx.x;
    const long long li = (long long)blockIdx.x * per + lane;
    unsigned nrot = 0;
    unsigned long long cols = 0;
    if (lane < per && li < nleaves) {
        const LeafRec L = leaves[li];
        const int st = body_leaf(L, d, e, pmax, w, out, sd + lane, se + lane, s0 + lane, s1 + lane, per, &nrot);
        if (st) atomicOr(w.status, st);
        cols = (unsigned long long)L.size;
    }
    // one atomic per wave for each counter (every lane reaches this point)
    count_add(w.counters, CNT_LEAF_COLS, cols);
    count_add(w.counters, CNT_LEAF_ROT, (unsigned long long)nrot);
}

// ---------------------------------------------------------------------------
// Merges inside one wave: the in-wave leaves and the levels of many small
// merges keep every level array in LDS, one lane per column or per root.
// ---------------------------------------------------------------------------
constexpr int kDcCols = kLeafMax;  // columns of one in-wave leaf
static_assert(kDcCols == 64, "one lane per column of an in-wave leaf");

// LDS of one in-wave level: 18 double arrays of kDcCols entries (21 with the
// node state), 7 int arrays of kDcCols (+1) entries and the level's merge
// records (at most kDcCols / 2: every merge has two or more columns).
template <bool Nodes>
struct WaveLds {
    double b[(Nodes ? 21 : 18) * kDcCols];
    int i[3 * kDcCols + 4 * (kDcCols + 1)];
    MergeRec smr[kDcCols / 2];
};

// Level arrays of an in-wave level in LDS.  A level runs merge | flags | runs |
// three-way split | roots | Loewner | rows | assembly; the merged and rotated
// columns (D, Z, RL, RH, D2, Z2) are last read by the split, so the later
// steps' arrays live in them: active z (split to Loewner) in Z, tau in D, the
// root values in D2, z-hat in Z2, the parent rows in RL and RH; the roots'
// origins reuse the candidate positions, last read by the runs.  Fewer arrays
// let more waves share a compute unit.  With Nodes, the node state lam, blo,
// bhi gets LDS storage too.
template <bool Nodes>
__device__ __forceinline__ void wave_arrays(WaveLds<Nodes>& sh, Work& wl) {
    constexpr int C = kDcCols;
    double* p = sh.b;
    if (Nodes) {
        wl.lam = p; p += C;  wl.blo = p; p += C;  wl.bhi = p; p += C;
    }
    wl.D = p; p += C;    wl.Z = p; p += C;    wl.RL = p; p += C;   wl.RH = p; p += C;
    wl.D2 = p; p += C;   wl.Z2 = p; p += C;   wl.RL2 = p; p += C;  wl.RH2 = p; p += C;
    wl.Da = p; p += C;   wl.Wa = p; p += C;   wl.RLa = p; p += C;  wl.RHa = p; p += C;
    wl.Dd = p; p += C;   wl.RLd = p; p += C;  wl.RHd = p; p += C;
    wl.Dr = p; p += C;   wl.RLr = p; p += C;  wl.RHr = p; p += C;
    wl.Za = wl.Z;        wl.tau = wl.D;       wl.rootval = wl.D2;  wl.zhat = wl.Z2;
    wl.PBL = wl.RL;      wl.PBH = wl.RH;
    int* q = sh.i;
    wl.src = q; q += C;  wl.nnpos = q; q += C;  wl.amerge = q; q += C;  wl.org = wl.nnpos;
    wl.st = q; q += C + 1;  wl.scan = q; q += C + 1;  wl.scanC = q; q += C + 1;  wl.scanR = q; q += C + 1;
}

// Work done by the in-wave levels of one wave (for the counters).
struct WaveCount {
    unsigned long long terms = 0, sweeps = 0, roots = 0, lpairs = 0, rpairs = 0, mcols = 0;
    int bad = 0;
};

// Roots, Loewner z and rows of an in-wave level with the canonical group sums
// of the whole-merge workgroups (defined with them below), G lanes per root.
template <int G>
__device__ void wave_roots_canon(const MergeRec* smr, int K, const double* __restrict__ e,
                                 const unsigned long long* __restrict__ pmax, const Work& wl,
                                 int* __restrict__ corg, double* __restrict__ ctau, long long pk0, WaveCount& c);

// One level of merges inside one wave: M merges (records in smr, pk local to
// the level arrays of wl), N columns in all, one lane per column or per active
// root.  Each merge runs the same per-column and per-root steps as the
// level-wide kernels (merged order and z~, negligible-z and close-pole
// deflation, secular roots, Loewner z, boundary rows, three-list assembly);
// only the compactions differ: a wave ballot replaces the block scans.  The
// children's spectra and rows are read through wl, the parents' are written
// through wl, or through wt when `top` (or the scaled eigenvalues to out for a
// problem's top merge).
// With corg, every root's origin and offset are also stored at the merge's
// packed position pk0 + smr[m].pk + (root index within the merge).  CG > 0:
// the root steps take CG lanes per root and the canonical group sums, so a
// level gives the same bits as in a whole-merge workgroup; CG = 0: one lane
// per root sums serially.
template <int CG>
__device__ __forceinline__ void wave_level(const MergeRec* smr, int M, int N, const double* __restrict__ e,
                                           const unsigned long long* __restrict__ pmax, const Work& wl,
                                           const Work& wt, bool top, double* __restrict__ out,
                                           int* __restrict__ corg, double* __restrict__ ctau, long long pk0,
                                           WaveCount& c) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    c.mcols += (lane == 0) ? (unsigned long long)N : 0ULL;
    // merged order, z~, negligible-z flags (lane = child column; its flag
    // lands with it at the merged position)
    if (lane < N) {
        int fl;
        body_merge(lane, find_merge(smr, M, lane), smr, e, pmax, wl, &fl);
    }
    __syncthreads();
    const int f = (lane < N) ? wl.st[lane] : 0;
    const unsigned long long cm = __ballot(f != 0);
    if (lane < N) {
        const int gc = (int)__popcll(cm & below);
        wl.scanC[lane] = gc;
        if (f) wl.nnpos[gc] = lane;
    }
    if (lane == 0) wl.scanC[N] = (int)__popcll(cm);
    __syncthreads();
    // close-pole runs
    if (lane < (int)__popcll(cm)) body_runs(lane, find_merge(smr, M, wl.nnpos[lane]), smr, wl, [](long long) {});
    __syncthreads();
    // three-way split
    const int s = (lane < N) ? wl.st[lane] : 0;
    const unsigned long long am = __ballot(lane < N && s == 1);
    const unsigned long long rm = __ballot(lane < N && s == 2);
    const int g = (int)__popcll(am & below), gr = (int)__popcll(rm & below);
    if (lane < N) {
        wl.scan[lane] = g;
        wl.scanR[lane] = gr;
        if (s == 1) {
            const double z = wl.Z2[lane];
            wl.Da[g] = wl.D2[lane];
            wl.Za[g] = z;
            wl.Wa[g] = z * z;
            wl.RLa[g] = wl.RL2[lane];
            wl.RHa[g] = wl.RH2[lane];
            wl.amerge[g] = find_merge(smr, M, lane);
        } else if (s == 2) {
            wl.Dr[gr] = wl.D2[lane];
            wl.RLr[gr] = wl.RL2[lane];
            wl.RHr[gr] = wl.RH2[lane];
        } else {
            const int q = lane - g - gr;
            wl.Dd[q] = wl.D[lane];
            wl.RLd[q] = wl.RL[lane];
            wl.RHd[q] = wl.RH[lane];
        }
    }
    if (lane == 0) {
        wl.scan[N] = (int)__popcll(am);
        wl.scanR[N] = (int)__popcll(rm);
    }
    __syncthreads();
    // secular roots, Loewner z, boundary rows
    const int K = (int)__popcll(am);
    if constexpr (CG > 0) {
        wave_roots_canon<CG>(smr, K, e, pmax, wl, corg, ctau, pk0, c);
        if (lane < N) body_assemble(lane, find_merge(smr, M, lane), smr, pmax, wl, out);
        __syncthreads();
        return;
    }
    // (one lane per active root)
    const int m = (lane < K) ? wl.amerge[lane] : 0;
    const bool rowsm = (lane < K) && (!(smr[m].flags & MF_ROOT) || wl.rows_out);
    int Km = 0;
    if (lane < K) {
        const MergeSpan sp = merge_span(smr[m], wl.scan);
        Km = sp.K;
        const int it = body_secular<RedSerial>(lane, m, smr, e, pmax, wl, 0, 1, wl.Da, wl.Wa, 0);
        if (it < 0) c.bad = 1;
        const unsigned long long sw = (Km > 1) ? (unsigned long long)((it < 0 ? wl.sec_cap : it) + 1) : 0ULL;
        c.terms += sw * (unsigned long long)Km;
        c.roots += 1;
        if (corg) {
            const long long gp = pk0 + smr[m].pk + (lane - sp.ks);
            corg[gp] = wl.org[lane];
            ctau[gp] = wl.tau[lane];
        }
    }
    __syncthreads();
    if (lane < K) body_lowner<RedSerial>(lane, m, smr, e, pmax, wl, 0, 1, wl.Da, wl.org, wl.tau, 0);
    __syncthreads();
    if (lane < K) body_rows<RedSerial>(lane, m, smr, wl, 0, 1, wl.Da, wl.zhat, wl.RLa, wl.RHa, 0);
    if (rowsm) {
        c.lpairs += (unsigned long long)Km;
        c.rpairs += (unsigned long long)Km;
    }
    __syncthreads();
    // parent spectra and rows (in place), or the problem's outputs
    if (lane < N) {
        if (top) body_assemble(lane, find_merge(smr, M, lane), smr, pmax, wt, out);
        else body_assemble(lane, find_merge(smr, M, lane), smr, pmax, wl, out);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Leaves solved by divide and conquer inside one wave (one workgroup of 64
// lanes per leaf of at most 64 columns).  The leaf's own merge tree (balanced
// halving down to single columns, Section 3.1; levelled by height) runs level
// by level with every level array in LDS (wave_level).  The leaf's top merge
// writes its node's spectrum and rows to the global arrays (or the scaled
// eigenvalues when the leaf is a whole problem).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_leaf_dc(const LeafRec* __restrict__ leaves,
                                               const SubHdr* __restrict__ shdr,
                                               const SubMerge* __restrict__ smer,
                                               const double* __restrict__ d, const double* __restrict__ e,
                                               const unsigned long long* __restrict__ pmax, Work w,
                                               double* __restrict__ out) {
    if (input_nonfinite(w)) return;
    __shared__ WaveLds<true> sh;
    const LeafRec L = leaves[blockIdx.x];
    const int l = L.size;
    const int lane = threadIdx.x;
    const double inv = 1.0 / scale_of(pmax[L.prob]);
    const double* eL = e + L.off;  // merge records below carry leaf-local offsets

    // level arrays and the node state (nodes that no merge of a level touches
    // carry their values to a higher level) in LDS
    Work wl = w;
    wave_arrays(sh, wl);
    // destinations of the leaf's top merge
    Work wt = wl;
    wt.lam = w.lam + L.off;
    wt.blo = w.blo + L.off;
    wt.bhi = w.bhi + L.off;
    wt.qfirst = w.qfirst ? w.qfirst + L.off : nullptr;
    wt.qlast = w.qlast ? w.qlast + L.off : nullptr;
    double* outL = out + L.off;

    // single-column nodes: the torn diagonal (every coupling inside the leaf is
    // torn, plus the leaf's own torn ends), first and last row 1
    if (lane < l) {
        double di = d[L.off + lane] * inv;
        if (lane > 0 || (L.flags & LF_TEAR_LEFT)) di -= fabs(eL[lane - 1] * inv);
        if (lane < l - 1 || (L.flags & LF_TEAR_RIGHT)) di -= fabs(eL[lane] * inv);
        if (l == 1) {
            if (L.flags & LF_WHOLE) {
                outL[0] = di / inv;
                if (w.rows_out) store_rows(wt, 0, 1.0, 1.0);
            } else {
                wt.lam[0] = di;
                wt.blo[0] = 1.0;
                wt.bhi[0] = 1.0;
            }
        }
        wl.lam[lane] = di;
        wl.blo[lane] = 1.0;
        wl.bhi[lane] = 1.0;
    }
    if (lane == 0) {
        count_add1(w.counters, CNT_LEAF_COLS, (unsigned long long)l);
    }
    if (l <= 1) return;
    const SubHdr* hd = shdr + l;  // read in place: a local copy of lv[] would live in scratch
    const int H = hd->H, mbase = hd->mbase;
    WaveCount c;
    for (int h = 0; h < H; ++h) {
        const int m0 = hd->lv[h];
        const int M = hd->lv[h + 1] - m0;
        const bool top = (h == H - 1);
        if (lane < M) {
            const SubMerge sm = smer[mbase + m0 + lane];
            MergeRec R;
            R.off = sm.off;
            R.pk = sm.pk;
            R.nL = sm.nL;
            R.nR = sm.nR;
            R.prob = L.prob;
            R.flags = (top && (L.flags & LF_WHOLE)) ? MF_ROOT : 0;
            sh.smr[lane] = R;
        }
        __syncthreads();
        const int N = (int)sh.smr[M - 1].pk + sh.smr[M - 1].nL + sh.smr[M - 1].nR;
        wave_level<0>(sh.smr, M, N, eL, pmax, wl, wt, top, outL, nullptr, nullptr, 0, c);
    }
    if (c.bad) atomicOr(w.status, ST_SEC_NOCONV);
    count_add(w.counters, CNT_DC_TERMS, c.terms);
    count_add(w.counters, CNT_DC_ROOTS, c.roots);
    count_add(w.counters, CNT_DC_LOW_PAIRS, c.lpairs);
    count_add(w.counters, CNT_DC_ROW_PAIRS, c.rpairs);
    count_add(w.counters, CNT_MERGE_COLS, c.mcols);
}

// ---------------------------------------------------------------------------
// Levels of many merges of at most kDcCols columns: one wave per pack of
// consecutive merges holding at most kDcCols columns in all (the plan's pack
// table: first merge of every pack, then the level's merge count), the level
// arrays in LDS as in the in-wave leaves, the children's spectra and rows read
// from the node arrays and the parents' written back in place.  A dependent
// chain of LDS steps per wave instead of global-memory round trips per step,
// and up to four small merges per wave instead of a mostly idle workgroup
// each.  With corg (a checkpointing forward), the roots land at the merges'
// packed positions as k_level_block stores them.  G lanes per root: one on
// levels of merges of at most 32 columns (a root's update costs more than its
// few terms there), four on merges of up to 64.
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_level_wave(const MergeRec* __restrict__ mr, const int* __restrict__ packs,
                                                  const double* __restrict__ e,
                                                  const unsigned long long* __restrict__ pmax, Work w,
                                                  double* __restrict__ out, int save_roots) {
    if (input_nonfinite(w)) return;
    __shared__ WaveLds<false> sh;
    const int lane = threadIdx.x;
    const int m0 = packs[blockIdx.x], M = packs[blockIdx.x + 1] - m0;
    const long long pk0 = mr[m0].pk;
    if (lane < M) {
        MergeRec R = mr[m0 + lane];
        R.pk -= pk0;
        sh.smr[lane] = R;
    }
    Work wl = w;
    wave_arrays(sh, wl);
    __syncthreads();
    const int N = (int)sh.smr[M - 1].pk + sh.smr[M - 1].nL + sh.smr[M - 1].nR;
    WaveCount c;
    wave_level<G>(sh.smr, M, N, e, pmax, wl, wl, false, out, save_roots ? w.org : nullptr,
                     save_roots ? w.tau : nullptr, pk0, c);
    if (c.bad) atomicOr(w.status, ST_SEC_NOCONV);
    // the whole-merge workgroups' counters (the same work, counted alike)
    count_add(w.counters, CNT_SEC_TERMS, c.terms);
    count_add(w.counters, CNT_SWEEPS, c.sweeps);
    count_add(w.counters, CNT_ROOTS, c.roots);
    count_add(w.counters, CNT_LOW_PAIRS, c.lpairs);
    count_add(w.counters, CNT_ROW_PAIRS, c.rpairs);
    count_add(w.counters, CNT_LB_TERMS, c.terms);
    count_add(w.counters, CNT_LB_LOW_PAIRS, c.lpairs);
    count_add(w.counters, CNT_LB_ROW_PAIRS, c.rpairs);
    count_add(w.counters, CNT_LB_ROOTS, c.roots);
    count_add(w.counters, CNT_MERGE_COLS, c.mcols);
}

// ---------------------------------------------------------------------------
// Level steps.  Element-parallel kernels find the merge of packed position t
// inside [blkm[t/kWG], blkm[t/kWG + 1]] (a static per-block table of the
// plan), so each lookup searches only the few merges a block touches.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int merge_of(const MergeRec* __restrict__ mr, const int* __restrict__ blkm, long long t) {
    const long long b = t / kWG;
    return find_merge_in(mr, blkm[b], blkm[b + 1], t);
}

// Sum of in[0..b) over the workgroup (every thread gets it): a block's own
// exclusive prefix of the per-block counts, when there are few blocks.
__device__ __forceinline__ int block_prefix(const int* __restrict__ in, int b, int* wsum) {
    int v = 0;
    for (int i = threadIdx.x; i < b; i += blockDim.x) v += in[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) wsum[wid] = v;
    __syncthreads();
    int t = 0;
    for (int i = 0; i < nw; ++i) t += wsum[i];
    __syncthreads();
    return t;
}

// Merged order, z~, outer rows and the negligible-z flag of every column;
// candidates are counted per block of merged positions (bsumA, zeroed once
// per pass), one atomic per distinct block among a wave's columns.
__global__ __launch_bounds__(kWG) void k_merge(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                               long long N, const double* __restrict__ e,
                                               const unsigned long long* __restrict__ pmax, Work w) {
    if (input_nonfinite(w)) return;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    int f = 0, pb = -1;
    if (t < N) pb = (int)(body_merge(t, merge_of(mr, blkm, t), mr, e, pmax, w, &f) / kWG);
    if (t == 0) count_add1(w.counters, CNT_MERGE_COLS, (unsigned long long)N);
    // one atomic per distinct position block among the wave's columns
    const int lane = threadIdx.x & 63;
    bool pending = pb >= 0;
    for (;;) {
        const unsigned long long pm = __ballot(pending);
        if (pm == 0ULL) break;
        const int leader = __ffsll((long long)pm) - 1;
        const int lpb = __shfl(pb, leader, 64);
        const bool mine = pending && (pb == lpb);
        const unsigned long long fm = __ballot(mine && f);
        if (lane == leader && fm) atomicAdd(&w.bsumA[lpb], (int)__popcll(fm));
        pending = pending && !mine;
    }
}

// The same by output position (merge path), for levels of large merges: block b writes packed positions
// [b kWG, (b+1) kWG).  For each merge piece the block covers, the co-ranks
// of the piece's two ends (how many left-child values precede them) are found
// cooperatively, half the block per end, 128 probes a round, so a merge of
// s columns needs about log_128(s) dependent global reads instead of log2(s)
// per column; the two child slices are then staged in LDS and every thread
// places its own position with a search inside them.  Ties go left first, as
// in body_merge.  The block's candidate count is added to bsumA[b].
//
// co-rank(p) = smallest i in [max(0, p - nR), min(p, nL)] with
// i == min(p, nL) or lamL[i] > lamR[p - i - 1].
__device__ __forceinline__ bool corank_pred(const double* __restrict__ lamL, const double* __restrict__ lamR,
                                            int p, int i, int hi) {
    return (i >= hi) || (lamL[i] > lamR[p - i - 1]);
}

__global__ __launch_bounds__(kWG) void k_merge_path(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                                    long long N, const double* __restrict__ e,
                                                    const unsigned long long* __restrict__ pmax, Work w) {
    if (input_nonfinite(w)) return;
    __shared__ double sL[kWG], sR[kWG];
    __shared__ int s_k[4];
    __shared__ int s_co[2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, half = tid >> 7, kt = tid & 127;
    const long long p0 = (long long)blockIdx.x * kWG;
    const long long p1 = (p0 + kWG < N) ? p0 + kWG : N;
    const long long P = p0 + tid;
    int f = 0;
    const int mfirst = blkm[blockIdx.x], mlast = blkm[blockIdx.x + 1];
    for (int m = mfirst; m <= mlast; ++m) {
        const MergeRec R = mr[m];
        const int s = R.nL + R.nR;
        const long long ga = (p0 > R.pk) ? p0 : R.pk;
        const long long gb = (p1 < R.pk + s) ? p1 : R.pk + s;
        if (ga >= gb) continue;  // block-uniform
        const int a = (int)(ga - R.pk), bnd = (int)(gb - R.pk);
        const double* lamL = w.lam + R.off;
        const double* lamR = lamL + R.nL;
        // co-ranks of a (first half) and bnd (second half)
        const int pe = half ? bnd : a;
        int lo = (pe - R.nR > 0) ? pe - R.nR : 0;
        int hi = (pe < R.nL) ? pe : R.nL;
        const int hi0 = hi;
        for (int round = 0; round < 8; ++round) {
            const bool active = hi > lo;
            if (!__syncthreads_or(active)) break;
            const int r = hi - lo;
            const int step = (r + 127) / 128;
            if (active) {
                const long long i = (long long)lo + (long long)kt * step;
                const bool t = (i >= hi) || corank_pred(lamL, lamR, pe, (int)i, hi0);
                const unsigned long long bm = __ballot(t);
                if (lane == 0) s_k[wv] = bm ? (wv & 1) * 64 + __ffsll((long long)bm) - 1 : 128;
            }
            __syncthreads();
            if (active) {
                const int k = min(s_k[2 * half], s_k[2 * half + 1]);
                const int nhi = (k < 128) ? lo + k * step : hi;
                const int nlo = (k == 0) ? lo : lo + (k - 1) * step + 1;
                lo = nlo;
                hi = nhi < hi ? nhi : hi;
            }
        }
        if (kt == 0) s_co[half] = lo;
        __syncthreads();
        const int ia = s_co[0], ib = s_co[1];
        const int ja = a - ia, jb = bnd - ib;
        // stage the two slices
        if (tid < ib - ia && ia + tid < R.nL) sL[tid] = lamL[ia + tid];
        if (tid < jb - ja && ja + tid < R.nR) sR[tid] = lamR[ja + tid];
        __syncthreads();
        const int p = (int)(P - R.pk);
        if (P >= ga && P < gb) {
            // co-rank of p inside the slices
            int l2 = (p - jb > ia) ? p - jb : ia;
            int h2 = (p - ja < ib) ? p - ja : ib;
            const int h20 = h2;
            while (l2 < h2) {
                const int mid = (l2 + h2) >> 1;
                if (mid >= h20 || sL[mid - ia] > sR[p - mid - 1 - ja]) h2 = mid;
                else l2 = mid + 1;
            }
            const int i = l2, j = p - i;
            const bool left = (i < ib) && (j >= jb || sL[i - ia] <= sR[j - ja]);
            double sgn;
            const double rho = merge_rho(R, e, pmax, &sgn);
            const double tol = merge_tol_children(R, w);
            const double x = left ? sL[i - ia] : sR[j - ja];
            f = merge_emit(R, left ? i : R.nL + j, x, rho, sgn, tol, w, P);
        }
        __syncthreads();  // slices and s_co are reused by the next piece
    }
    const int cnt = __syncthreads_count(f);
    if (tid == 0 && cnt) atomicAdd(&w.bsumA[blockIdx.x], cnt);
    if (P == 0) count_add1(w.counters, CNT_MERGE_COLS, (unsigned long long)N);
}

// Compaction of candidate (st == 1) columns: scanC[t] = exclusive count,
// nnpos[g] = t for the g-th candidate.  The block's base is its own prefix of
// the block counts (selfscan) or the scanned counts in bsum.
__global__ __launch_bounds__(kWG) void k_nncompact(long long N, Work w, int selfscan) {
    if (input_nonfinite(w)) return;
    __shared__ int wsum[16];
    const int base = selfscan ? block_prefix(w.bsumA, blockIdx.x, wsum) : w.bsum[blockIdx.x];
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int f = (t < N) ? (w.st[t] == 1) : 0;
    const int incl = block_incl_scan(f, wsum);
    const int g = base + incl - f;
    if (t < N) {
        w.scanC[t] = g;
        if (f && g < N) w.nnpos[g] = (int)t;
        if (t == N - 1) w.scanC[N] = g + f;
    }
}

// Close-pole runs over the candidates (grid-stride).  Each rotated-away
// column moves one count from its block's active tally to its rotated tally.
__global__ __launch_bounds__(kWG) void k_runs(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                              long long N, Work w) {
    if (input_nonfinite(w)) return;
    const long long total = min((long long)w.scanC[N], N);
    int* bA = w.bsumA;
    int* bR = w.bsumR;
    auto on_rotate = [bA, bR](long long p) {
        atomicSub(&bA[p / kWG], 1);
        atomicAdd(&bR[p / kWG], 1);
    };
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x)
        body_runs(g, merge_of(mr, blkm, w.nnpos[g]), mr, w, on_rotate);
}

// Three-way split of a level's columns: active ones to (Da, Za, RLa, RHa) at
// their active index, rotated-away ones to (Dr, RLr, RHr) and negligible-z
// ones to (Dd, RLd, RHd), each list in column order.  scan / scanR hold the
// exclusive active / rotated counts.  Candidates read their post-rotation
// values (D2, ...), negligible columns the merged ones (D, ...).
__global__ __launch_bounds__(kWG) void k_actcompact(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                                    long long N, Work w, int selfscan) {
    if (input_nonfinite(w)) return;
    __shared__ int wsum[16];
    int baseA, baseR;
    if (selfscan) {
        baseA = block_prefix(w.bsumA, blockIdx.x, wsum);
        baseR = block_prefix(w.bsumR, blockIdx.x, wsum);
    } else {
        baseA = w.bsumAs[blockIdx.x];
        baseR = w.bsumRs[blockIdx.x];
    }
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int s = (t < N) ? w.st[t] : 0;
    const int fa = (t < N) && (s == 1);
    const int fr = (t < N) && (s == 2);
    const int ia = block_incl_scan(fa, wsum);
    __syncthreads();
    const int ir = block_incl_scan(fr, wsum);
    const int g = baseA + ia - fa;
    const int gr = baseR + ir - fr;
    if (t < N) {
        w.scan[t] = g;
        w.scanR[t] = gr;
        if (fa && g < N) {
            w.Da[g] = w.D2[t];
            w.Za[g] = w.Z2[t];
            w.Wa[g] = w.Z2[t] * w.Z2[t];
            w.RLa[g] = w.RL2[t];
            w.RHa[g] = w.RH2[t];
            w.amerge[g] = merge_of(mr, blkm, t);
            w.apos[g] = (int)t;
        } else if (fr && gr < N) {
            w.Dr[gr] = w.D2[t];
            w.RLr[gr] = w.RL2[t];
            w.RHr[gr] = w.RH2[t];
            w.rpos[gr] = (int)t;
        } else if (!fa && !fr && t - g - gr >= 0 && t - g - gr < N) {
            const long long q = t - g - gr;
            w.Dd[q] = w.D[t];
            w.RLd[q] = w.RL[t];
            w.RHd[q] = w.RH[t];
            w.dpos[q] = (int)t;
        }
        if (t == N - 1) {
            w.scan[N] = g + fa;
            w.scanR[N] = gr + fr;
        }
    }
}

// Group reduction over G <= 16 consecutive lanes with DPP lane moves (no LDS
// crossbar): swap within pairs, then within quads, then mirror the
// eight-lane half rows, then the sixteen-lane rows.  Each step pairs lane i
// with a partner that takes lane i as its own partner, and x + y == y + x
// bit for bit, so every lane of the group ends with the same bits.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr int kDppSwap1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within eight lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within sixteen lanes

template <int G>
struct RedGroup {
    static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group of 2..16 lanes");
    __device__ __forceinline__ static double sum(double x) {
        x += dpp_move<kDppSwap1>(x);
        if (G >= 4) x += dpp_move<kDppSwap2>(x);
        if (G >= 8) x += dpp_move<kDppHalfMirror>(x);
        if (G >= 16) x += dpp_move<kDppMirror>(x);
        return x;
    }
    __device__ __forceinline__ static double prod(double x) {
        x *= dpp_move<kDppSwap1>(x);
        if (G >= 4) x *= dpp_move<kDppSwap2>(x);
        if (G >= 8) x *= dpp_move<kDppHalfMirror>(x);
        if (G >= 16) x *= dpp_move<kDppMirror>(x);
        return x;
    }
};
template <>
struct RedGroup<1> {
    __device__ __forceinline__ static double sum(double x) { return x; }
    __device__ __forceinline__ static double prod(double x) { return x; }
};

// Root-parallel steps: a group of G lanes per root (or per pole for the
// Loewner step).  A workgroup takes tiles of kWG/G consecutive active columns;
// when the merges covering a tile hold at most kStage active columns, their
// arrays are first staged in LDS and every sweep reads them from there.
constexpr int kStage = 2048;
constexpr int kStageRows = 1024;

struct TileWindow {
    long long r0, r1;  // staged range of active columns
    bool staged;
};

__device__ __forceinline__ TileWindow tile_window(long long g0, long long g1, const MergeRec* __restrict__ mr,
                                                  const Work& w, int cap) {
    // g0 <= g1 < total: first and last active column of the tile
    const int m0 = w.amerge[g0], m1 = w.amerge[g1];
    TileWindow tw;
    tw.r0 = w.scan[mr[m0].pk];
    tw.r1 = w.scan[mr[m1].pk + mr[m1].nL + mr[m1].nR];
    tw.staged = (tw.r1 - tw.r0) <= cap;
    return tw;
}

// ---------------------------------------------------------------------------
// Wide sweeps for merges with many active roots (K >= wide_min).  A
// workgroup takes 64 consecutive roots (or poles) of one merge, one per lane;
// its kWideWaves waves split the other index into segments.  Within a wave
// that index is uniform, so the per-pole (per-root) operands are scalar loads
// shared by the 64 lanes, and the left/right split and the origin exclusion
// of the secular sums become loop bounds: only the window next to the
// block's own roots needs per-lane selects.  The waves' partial results meet
// in LDS in a fixed order, so every wave holds the same totals bit for bit.
// The wide blocks are the trailing blocks of the regular root kernels'
// grids (block-uniform split); the work items (64-root blocks of the wide
// merges) are listed once per level by k_wide_items.
// ---------------------------------------------------------------------------
static_assert(64 * kWideWaves == kWG, "wide blocks share the regular kernels' workgroup size");
static_assert(2 * 5 * kWideWaves * 64 <= 2 * 2048, "wide reduction buffers fit the regular kernels' LDS staging area");

// Exclusive scan of the number of 64-root blocks of every wide merge of a level.
__global__ __launch_bounds__(1024) void k_wide_items(const MergeRec* __restrict__ mr, int M, Work w, int wide_min,
                                                     int fuse_max) {
    if (input_nonfinite(w)) return;
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < M; base += 1024) {
        const int m = base + threadIdx.x;
        int v = 0;
        if (m < M) {
            const int K = merge_span(mr[m], w.scan).K;
            v = (K >= wide_min && K > fuse_max) ? (K + 63) / 64 : 0;
        }
        const int incl = block_incl_scan(v, wsum);
        const int c = carry;
        if (m < M) w.witems[m] = c + incl - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = c + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) w.witems[M] = carry;
}

// Values the compiler cannot prove wave-uniform but are (the wave index, a
// merge's offsets): moved to scalar registers so the loops over them use
// scalar loads.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long wave_uniform(long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Merge owning wide item `item` (largest m with witems[m] <= item), uniform.
__device__ __forceinline__ int wide_merge_of(const int* witems, int M, int item) {
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (witems[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

struct WideSums {
    double ps, dps, ph, dph, zz;
};

// Read-only views in the constant address space: a wave-uniform index into
// them is a scalar load (s_load through the scalar data cache; these arrays
// are written only by earlier launches, and nothing here is ever stored
// through that cache).
typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) int cint;
__device__ __forceinline__ cdouble* as_const(const double* p) { return (cdouble*)p; }
__device__ __forceinline__ cint* as_const(const int* p) { return (cint*)p; }

// Secular sums over poles j in [a, b) (wave-uniform) for this lane's root:
// left poles j < L1 into (ps, dps), right poles j >= R0 into (ph, dph); poles
// in [L1, R0) are skipped.  [w0, w1) (wave-uniform) contains every lane's
// [L1, R0); below it every pole is left for every lane, above it right.
template <bool ZZ>
__device__ __forceinline__ void wide_sweep(cdouble* D, cdouble* W, int a, int b, int w0, int w1, double Do, double tau,
                                           int L1, int R0, WideSums& s) {
    const int e1 = min(b, w0);
    _Pragma("unroll 4") for (int j = a; j < e1; ++j) {
        const double r = rcp_nr((D[j] - Do) - tau);
        const double t = W[j] * r;
        s.ps += t;
        s.dps = fma(t, r, s.dps);
        if (ZZ) s.zz += W[j];
    }
    const int s2 = max(a, w0), e2 = min(b, w1);
    for (int j = s2; j < e2; ++j) {
        const double r = rcp_nr((D[j] - Do) - tau);
        const double t = W[j] * r;
        const double dt = t * r;
        const bool lf = j < L1, rt = j >= R0;
        s.ps += lf ? t : 0.0;
        s.dps += lf ? dt : 0.0;
        s.ph += rt ? t : 0.0;
        s.dph += rt ? dt : 0.0;
        if (ZZ) s.zz += W[j];
    }
    _Pragma("unroll 4") for (int j = max(a, w1); j < b; ++j) {
        const double r = rcp_nr((D[j] - Do) - tau);
        const double t = W[j] * r;
        s.ph += t;
        s.dph = fma(t, r, s.dph);
        if (ZZ) s.zz += W[j];
    }
}

// Wide secular roots with NW waves per block.  red: 2 x 5 x NW x 64 doubles
// of LDS.  The block iterates until all of its 64 roots have converged.
template <int NW>
__device__ void secular_wide(int bid, int nbw, const MergeRec* __restrict__ mr, int M, const double* __restrict__ e,
                             const unsigned long long* __restrict__ pmax, const Work& w, const int* items,
                             double* red) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform((int)(threadIdx.x >> 6));
    auto R5 = [&](int buf, int q, int v) -> double& { return red[((buf * 5 + q) * NW + v) * 64 + lane]; };
    const int total = items[M];
    int buf = 0;
    int bad = 0;
    unsigned long long terms = 0, sweeps = 0, roots = 0;
    for (int item = bid; item < total; item += nbw) {
        const int m = wide_merge_of(items, M, item);
        const MergeRec R = mr[m];
        const MergeSpan sp = merge_span(R, w.scan);
        const int K = wave_uniform(sp.K);
        const long long ks = wave_uniform(sp.ks);
        const int k0 = __builtin_amdgcn_readfirstlane((item - items[m]) * 64);
        const double* D = w.Da + ks;
        const double* Z = w.Za + ks;
        cdouble* Dc = as_const(D);
        cdouble* Wc = as_const(w.Wa + ks);
        double sgn;
        const double rho = merge_rho(R, e, pmax, &sgn);
        const int k = min(k0 + lane, K - 1);
        const bool act = (k0 + lane) < K;
        const int kk = min(k, K - 2);
        const int klast = min(k0 + 63, K - 1);
        const int w0 = k0, w1 = min(min(klast, K - 2) + 2, K);
        const int a = (int)((long long)K * wv / NW), b = (int)((long long)K * (wv + 1) / NW);
        // first sweep: bracket midpoint with origin kk (the last root also needs ||z||^2)
        WideSums s{0.0, 0.0, 0.0, 0.0, 0.0};
        wide_sweep<true>(Dc, Wc, a, b, w0, w1, D[kk], 0.5 * (D[kk + 1] - D[kk]), kk, kk + 2, s);
        double tot[5];
        R5(buf, 0, wv) = s.ps;
        R5(buf, 1, wv) = s.dps;
        R5(buf, 2, wv) = s.ph;
        R5(buf, 3, wv) = s.dph;
        R5(buf, 4, wv) = s.zz;
        __syncthreads();
        for (int q = 0; q < 5; ++q) {
            double x = 0.0;
            for (int v = 0; v < NW; ++v) x += R5(buf, q, v);
            tot[q] = x;
        }
        buf ^= 1;
        SecRoot r;
        bool done;
        if (k < K - 1) {
            done = sec_start_interior(k, D, Z, rho, tot[0], tot[1], tot[2], tot[3], &r);
        } else {
            sec_start_last(K, D, Z, rho, tot[4], &r);
            done = false;
        }
        int its = 0;
        for (int it = 1; it <= w.sec_cap; ++it) {
            if (__all(done)) break;
            const int L1 = r.orgl ? kk : kk + 1;
            const int R0 = r.orgl ? kk + 1 : kk + 2;
            WideSums u{0.0, 0.0, 0.0, 0.0, 0.0};
            wide_sweep<false>(Dc, Wc, a, b, w0, w1, D[r.o], r.tau, L1, R0, u);
            R5(buf, 0, wv) = u.ps;
            R5(buf, 1, wv) = u.dps;
            R5(buf, 2, wv) = u.ph;
            R5(buf, 3, wv) = u.dph;
            __syncthreads();
            for (int q = 0; q < 4; ++q) {
                double x = 0.0;
                for (int v = 0; v < NW; ++v) x += R5(buf, q, v);
                tot[q] = x;
            }
            buf ^= 1;
            if (!done && sec_update(&r, rho, tot[0], tot[1], tot[2], tot[3], tot[2] - tot[0])) {
                done = true;
                its = it;
            }
        }
        if (!done) bad = 1;
        if (wv == 0 && act) {
            w.org[ks + k] = r.o;
            w.tau[ks + k] = r.tau;
            const double dor = D[r.o];
            w.dorg[ks + k] = dor;
            w.rootval[ks + k] = dor + r.tau;
            const unsigned long long sw = (unsigned long long)((done ? its : w.sec_cap) + 1);
            sweeps += sw;
            terms += sw * (unsigned long long)K;
            roots += 1;
        }
        __syncthreads();
    }
    if (bad && wv == 0 && lane == 0) atomicOr(w.status, ST_SEC_NOCONV);
    if (wv == 0) {
        count_add(w.counters, CNT_SEC_TERMS, terms);
        count_add(w.counters, CNT_SWEEPS, sweeps);
        count_add(w.counters, CNT_ROOTS, roots);
    }
}

// Wide Loewner step: 64 poles per workgroup, the roots split over the waves
// (root index wave-uniform: D_org, tau and the neighbouring poles are scalar
// loads).  Factors are multiplied in chunks of 8 numerators and 8
// denominators, one division per chunk.  red: NW x 64 doubles.  DORG: take
// D_org of each root from w.dorg (written by secular_wide in the same
// forward level) instead of gathering D[org[k]], so the scalar loads of one
// factor do not wait on each other.
template <int NW, bool DORG>
__device__ void lowner_wide(int bid, int nbw, const MergeRec* __restrict__ mr, int M, const double* __restrict__ e,
                            const unsigned long long* __restrict__ pmax, const Work& w, bool with_root,
                            const int* items, double* red) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform((int)(threadIdx.x >> 6));
    const int total = items[M];
    unsigned long long pairs = 0;
    for (int item = bid; item < total; item += nbw) {
        const int m = wide_merge_of(items, M, item);
        const MergeRec R = mr[m];
        if (!(R.flags & MF_ROOT) || with_root || w.rows_out) {
            const MergeSpan sp = merge_span(R, w.scan);
            const int K = wave_uniform(sp.K);
            const long long ks = wave_uniform(sp.ks);
            const int i0 = __builtin_amdgcn_readfirstlane((item - items[m]) * 64);
            cdouble* D = as_const(w.Da + ks);
            cint* og = as_const(w.org + ks);
            cdouble* dg = as_const(w.dorg + ks);
            cdouble* ta = as_const(w.tau + ks);
            auto dorg = [&](int k) -> double { return DORG ? dg[k] : D[og[k]]; };
            const int i = min(i0 + lane, K - 1);
            const double di = w.Da[ks + i];
            const int ilast = min(i0 + 63, K - 1);
            const int a = (int)((long long)K * wv / NW), b = (int)((long long)K * (wv + 1) / NW);
            double prod = 1.0, pn = 1.0, pd = 1.0;
            int c = 0;
            auto factor = [&](double num, double den) {
                pn *= num;
                pd *= den;
                if (++c == 8) {
                    prod *= pn / pd;
                    pn = 1.0;
                    pd = 1.0;
                    c = 0;
                }
            };
            // k < i0: every lane has k < i
            const int e1 = min(b, i0);
            for (int k = a; k < e1; ++k) factor((dorg(k) - di) + ta[k], D[k] - di);
            // window: k in [i0, ilast]
            const int s2 = max(a, i0), e2 = min(b, ilast + 1);
            for (int k = s2; k < e2; ++k) {
                const double num = (dorg(k) - di) + ta[k];
                const double den = (k < i) ? D[k] - di : ((k < K - 1) ? D[k + 1] - di : 1.0);
                factor(num, den);
            }
            // ilast < k < K-1: every lane has i <= k
            const int e3 = min(b, K - 1);
            for (int k = max(a, ilast + 1); k < e3; ++k) factor((dorg(k) - di) + ta[k], D[k + 1] - di);
            if (b == K && ilast + 1 <= K - 1) factor((dorg(K - 1) - di) + ta[K - 1], 1.0);
            prod *= pn / pd;
            red[wv * 64 + lane] = prod;
            __syncthreads();
            if (wv == 0 && i0 + lane < K) {
                double p = 1.0;
                for (int v = 0; v < NW; ++v) p *= red[v * 64 + lane];
                double sgn;
                const double rho = merge_rho(R, e, pmax, &sgn);
                const double zi = sqrt(fmax(p / rho, 0.0));
                w.zhat[ks + i] = (w.Za[ks + i] < 0.0) ? -zi : zi;
                if (!(R.flags & MF_ROOT) || w.rows_out) pairs += (unsigned long long)K;
            }
        }
        __syncthreads();
    }
    if (wv == 0) count_add(w.counters, CNT_LOW_PAIRS, pairs);
}

// Wide boundary-row step (non-top merges): 64 roots per workgroup, the poles
// split over the waves, pole index wave-uniform (scalar loads of D_i, zhat_i
// and both row entries); no pole is excluded, so there is no window.
// red: 3 x NW x 64 doubles.
template <int NW>
__device__ void rows_wide(int bid, int nbw, const MergeRec* __restrict__ mr, int M, const Work& w, const int* items,
                          double* red) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform((int)(threadIdx.x >> 6));
    const int total = items[M];
    unsigned long long pairs = 0;
    for (int item = bid; item < total; item += nbw) {
        const int m = wide_merge_of(items, M, item);
        const MergeRec R = mr[m];
        if (!(R.flags & MF_ROOT) || w.rows_out) {
            const MergeSpan sp = merge_span(R, w.scan);
            const int K = wave_uniform(sp.K);
            const long long ks = wave_uniform(sp.ks);
            const int k0 = __builtin_amdgcn_readfirstlane((item - items[m]) * 64);
            cdouble* D = as_const(w.Da + ks);
            cdouble* H = as_const(w.zhat + ks);
            cdouble* RL = as_const(w.RLa + ks);
            cdouble* RH = as_const(w.RHa + ks);
            const int k = min(k0 + lane, K - 1);
            const double Do = w.Da[ks + w.org[ks + k]], tau = w.tau[ks + k];
            const int a = (int)((long long)K * wv / NW), b = (int)((long long)K * (wv + 1) / NW);
            double ss = 0.0, bl = 0.0, bh = 0.0;
            _Pragma("unroll 4") for (int i = a; i < b; ++i) {
                const double y = H[i] * rcp_nr((D[i] - Do) - tau);
                ss = fma(y, y, ss);
                bl = fma(RL[i], y, bl);
                bh = fma(RH[i], y, bh);
            }
            red[(0 * NW + wv) * 64 + lane] = ss;
            red[(1 * NW + wv) * 64 + lane] = bl;
            red[(2 * NW + wv) * 64 + lane] = bh;
            __syncthreads();
            if (wv == 0 && k0 + lane < K) {
                double t0 = 0.0, t1 = 0.0, t2 = 0.0;
                for (int v = 0; v < NW; ++v) {
                    t0 += red[(0 * NW + v) * 64 + lane];
                    t1 += red[(1 * NW + v) * 64 + lane];
                    t2 += red[(2 * NW + v) * 64 + lane];
                }
                const double inv = 1.0 / sqrt(t0);
                w.PBL[ks + k] = t1 * inv;
                w.PBH[ks + k] = t2 * inv;
                pairs += (unsigned long long)K;
            }
        }
        __syncthreads();
    }
    if (wv == 0) count_add(w.counters, CNT_ROW_PAIRS, pairs);
}

// Root-parallel kernels.  Blocks [0, nbn) take tiles of consecutive active
// columns of the merges below wide_min (G lanes per root); blocks from nbn on
// run the wide sweeps.
//
// Secular roots converge in different numbers of sweeps, so a group of G
// lanes does not wait for the slowest root of its wave or workgroup: each
// tile holds kRefill roots per group, and a group takes the next unsolved
// root of its tile (a workgroup counter in LDS) as soon as its current one
// has converged.  Every sweep, the bracket-midpoint one included, is the same
// sec_sweep call with per-group parameters, so groups in different phases
// still run one instruction stream.  Which group solves which root does not
// change any result.  The roots per group (refill, 1..4) are chosen per level
// so that the level still has about kRefillLanes lanes: refill only pays when
// the level has far more roots than the GPU has lanes (large batches).
constexpr int kRefillMax = 4;
constexpr long long kRefillLanes = 1048576;

// One merge of at most fuse_max (<= kFoldCap) active roots solved whole by a
// workgroup of NT threads (roots, Loewner z, rows), staged in `stage`.
constexpr int kFoldCap = 64;
template <int NT>
__device__ void small_merge_fold(int m, const MergeRec* __restrict__ mr, const double* __restrict__ e,
                                 const unsigned long long* __restrict__ pmax, const Work& w, int gmax, int fuse_max,
                                 double* stage, double* out, int amode);

template <int G>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) void k_secular(
    const MergeRec* __restrict__ mr, int M, long long N, const double* __restrict__ e,
    const unsigned long long* __restrict__ pmax, Work w, int wide_min, int fuse_max, int nbn, int refill, int nsm,
    int gmax, double* __restrict__ out, int amode) {
    if (input_nonfinite(w)) return;
    __shared__ double smem[2 * kStage];
    __shared__ long long s_r0;
    __shared__ int s_staged;
    __shared__ int s_next;
    // the last nsm workgroups solve the level's small merges whole (one each;
    // the tiles skip them), beside the tiles instead of in a launch of their own
    const int nbt = (int)gridDim.x - nsm;
    if ((int)blockIdx.x >= nbt) {
        small_merge_fold<kWG>((int)blockIdx.x - nbt, mr, e, pmax, w, gmax, fuse_max, smem, out, amode);
        return;
    }
    if ((int)blockIdx.x >= nbn) {
        const int* items = w.witems;
        secular_wide<kWideWaves>((int)blockIdx.x - nbn, nbt - nbn, mr, M, e, pmax, w, items, smem);
        return;
    }
    double* sD = smem;
    double* sW = smem + kStage;
    const long long total = min((long long)w.scan[N], N);
    const int T = (kWG / G) * refill;
    const int sub = threadIdx.x % G;
    int bad = 0;
    unsigned long long terms = 0, sweeps = 0, roots = 0;
    if (refill == 1) {
        // one root per group: the plain tile loop
        for (long long tile = blockIdx.x; tile * T < total; tile += nbn) {
            const long long g0 = tile * T;
            const long long g1 = (g0 + T < total ? g0 + T : total) - 1;
            if (threadIdx.x == 0) {
                const TileWindow tw = tile_window(g0, g1, mr, w, kStage);
                s_r0 = tw.r0;
                s_staged = tw.staged ? (int)(tw.r1 - tw.r0) : -1;
            }
            __syncthreads();
            const long long r0 = s_r0;
            const int ns = s_staged;
            if (ns >= 0)
                for (int i = threadIdx.x; i < ns; i += kWG) {
                    sD[i] = w.Da[r0 + i];
                    sW[i] = w.Wa[r0 + i];
                }
            __syncthreads();
            const long long g = g0 + threadIdx.x / G;
            const int mg = (g < total) ? w.amerge[g] : 0;
            const int Kg = (g < total) ? merge_span(mr[mg], w.scan).K : 0;
            if (g < total && Kg < wide_min && Kg > fuse_max) {
                const int it = (ns >= 0) ? body_secular<RedGroup<G>>(g, mg, mr, e, pmax, w, sub, G, sD, sW, r0)
                                         : body_secular<RedGroup<G>>(g, mg, mr, e, pmax, w, sub, G, w.Da, w.Wa, 0);
                if (it < 0) bad = 1;
                if (sub == 0) {
                    const MergeSpan sp = merge_span(mr[mg], w.scan);
                    const unsigned long long sw =
                        (sp.K > 1) ? (unsigned long long)((it < 0 ? w.sec_cap : it) + 1) : 0ULL;
                    sweeps += sw;
                    terms += sw * (unsigned long long)sp.K;
                    roots += 1;
                }
            }
            __syncthreads();
        }
    }
    for (long long tile = blockIdx.x; refill > 1 && tile * T < total; tile += nbn) {
        const long long g0 = tile * T;
        const long long g1 = (g0 + T < total ? g0 + T : total) - 1;
        if (threadIdx.x == 0) {
            const TileWindow tw = tile_window(g0, g1, mr, w, kStage);
            s_r0 = tw.r0;
            s_staged = tw.staged ? (int)(tw.r1 - tw.r0) : -1;
            s_next = 0;
        }
        __syncthreads();
        const long long r0 = s_r0;
        const int ns = s_staged;
        if (ns >= 0)
            for (int i = threadIdx.x; i < ns; i += kWG) {
                sD[i] = w.Da[r0 + i];
                sW[i] = w.Wa[r0 + i];
            }
        __syncthreads();
        // per-group state (every lane of a group holds the same copy)
        long long g = -1, ks = 0;
        int k = 0, K = 0, kk = 0, it = 0, phase = 0;
        double rho = 0.0;
        const double* Dv = nullptr;
        const double* Wv = nullptr;
        const double* Zg = nullptr;
        SecRoot r{};
        for (;;) {
            if (g < 0) {
                int slot = 0;
                if (sub == 0) slot = atomicAdd(&s_next, 1);
                slot = __shfl(slot, 0, G);
                if (g0 + slot > g1) break;
                g = g0 + slot;
                const MergeRec R = mr[w.amerge[g]];
                const MergeSpan sp = merge_span(R, w.scan);
                if (sp.K >= wide_min || sp.K <= fuse_max) {  // solved by the wide blocks or k_small_merge
                    g = -1;
                    continue;
                }
                K = sp.K;
                ks = sp.ks;
                k = (int)(g - ks);
                kk = (k < K - 1) ? k : K - 2;
                double sgn;
                rho = merge_rho(R, e, pmax, &sgn);
                Dv = (ns >= 0) ? sD + (ks - r0) : w.Da + ks;
                Wv = (ns >= 0) ? sW + (ks - r0) : w.Wa + ks;
                Zg = w.Za + ks;
                if (K == 1) {
                    if (sub == 0) {
                        w.org[g] = 0;
                        w.tau[g] = rho * Zg[0] * Zg[0];
                        w.rootval[g] = Dv[0] + w.tau[g];
                        roots += 1;
                    }
                    g = -1;
                    continue;
                }
                phase = 1;
                it = 0;
            }
            double Do, tau;
            int L1, R0;
            if (phase == 1) {  // bracket midpoint with origin kk (the last root uses only the weight sum)
                Do = Dv[kk];
                tau = 0.5 * (Dv[kk + 1] - Dv[kk]);
                L1 = kk;
                R0 = kk + 2;
            } else {
                Do = Dv[r.o];
                tau = r.tau;
                sec_split(r, kk, &L1, &R0);
            }
            double sm[5];
            sec_sweep<RedGroup<G>, true>(K, Dv, Wv, Do, tau, L1, R0, sub, G, sm);
            bool done = false;
            int used = 0;
            if (phase == 1) {
                if (k < K - 1) done = sec_start_interior(k, Dv, Zg, rho, sm[0], sm[1], sm[2], sm[3], &r);
                else sec_start_last(K, Dv, Zg, rho, sm[4], &r);
                phase = 2;
            } else {
                ++it;
                if (sec_update(&r, rho, sm[0], sm[1], sm[2], sm[3], sm[2] - sm[0])) {
                    done = true;
                    used = it;
                } else if (it >= w.sec_cap) {
                    done = true;
                    used = w.sec_cap;
                    bad = 1;
                }
            }
            if (done) {
                if (sub == 0) {
                    w.org[g] = r.o;
                    w.tau[g] = r.tau;
                    w.rootval[g] = Dv[r.o] + r.tau;
                    sweeps += (unsigned long long)(used + 1);
                    terms += (unsigned long long)(used + 1) * (unsigned long long)K;
                    roots += 1;
                }
                g = -1;
            }
        }
        __syncthreads();
    }
    if (bad && sub == 0) atomicOr(w.status, ST_SEC_NOCONV);
    count_add(w.counters, CNT_SEC_TERMS, terms);
    count_add(w.counters, CNT_SWEEPS, sweeps);
    count_add(w.counters, CNT_ROOTS, roots);
}

// Wide roots of a level on which every merge too large for k_small_merge is
// wide (no regular tiles): eight waves per 64-root block instead of four, so
// each wave sweeps an eighth of the poles and twice as many waves per SIMD
// hide the latency of the per-term chains.
// On levels of at most kWideOwnItems merges every block scans the merges' wide
// item counts itself (the work of k_wide_items, one launch less per level)
// and block 0 stores the table for the Loewner and row steps.
constexpr int kWideWavesOnly = 8;
constexpr int kWideOwnItems = 1024;
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_secular_wide(const MergeRec* __restrict__ mr, int M,
                                                          const double* __restrict__ e,
                                                          const unsigned long long* __restrict__ pmax, Work w,
                                                          int wide_min, int fuse_max, int own_items) {
    if (input_nonfinite(w)) return;
    __shared__ double red[2 * 5 * NW * 64];
    __shared__ int sitems[kWideOwnItems + 1];
    __shared__ int wsum[16];
    __shared__ int carry;
    const int* items = w.witems;
    if (own_items) {  // M <= kWideOwnItems (block-uniform)
        if (threadIdx.x == 0) carry = 0;
        __syncthreads();
        for (int base = 0; base < M; base += NW * 64) {
            const int m = base + (int)threadIdx.x;
            int v = 0;
            if (m < M) {
                const int K = merge_span(mr[m], w.scan).K;
                v = (K >= wide_min && K > fuse_max) ? (K + 63) / 64 : 0;
            }
            const int incl = block_incl_scan(v, wsum);
            const int c = carry;
            if (m < M) sitems[m] = c + incl - v;
            __syncthreads();
            if (threadIdx.x == NW * 64 - 1) carry = c + incl;
            __syncthreads();
        }
        if (threadIdx.x == 0) sitems[M] = carry;
        __syncthreads();
        if (blockIdx.x == 0)
            for (int m = threadIdx.x; m <= M; m += NW * 64) w.witems[m] = sitems[m];
        items = sitems;
    }
    secular_wide<NW>((int)blockIdx.x, (int)gridDim.x, mr, M, e, pmax, w, items, red);
}

// The same for the Loewner step and the rows (forward pass).
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_lowner_wide(const MergeRec* __restrict__ mr, int M,
                                                         const double* __restrict__ e,
                                                         const unsigned long long* __restrict__ pmax, Work w) {
    if (input_nonfinite(w)) return;
    __shared__ double red[NW * 64];
    lowner_wide<NW, true>((int)blockIdx.x, (int)gridDim.x, mr, M, e, pmax, w, false, w.witems, red);
}
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_rows_wide(const MergeRec* __restrict__ mr, int M, Work w) {
    if (input_nonfinite(w)) return;
    __shared__ double red[3 * NW * 64];
    rows_wide<NW>((int)blockIdx.x, (int)gridDim.x, mr, M, w, w.witems, red);
}

// ---------------------------------------------------------------------------
// Merges with at most kFuseMax active roots (after deflation): one workgroup
// of kFuseThreads (2 kFuseThreads on levels of merges of kFuseWideS columns
// or more) per merge runs the secular roots, the Loewner z and the boundary
// rows with the merge's active arrays staged in LDS once, with
// G = min(16, 2 kFuseThreads / K) lanes per root or pole rounded down to a
// power of two (the same device functions as the level-wide kernels, which
// skip these merges).  G depends on K alone, so a merge's arithmetic does not
// depend on the rest of its level (a batched solve matches the single ones
// bit for bit).  On random spectra nearly every merge is of this kind (a
// hundred or so roots survive deflation).
// ---------------------------------------------------------------------------
constexpr int kFuseMax = kFuseMaxRoots;
constexpr int kFuseThreads = 512;
constexpr int kFuseWideS = 2048;


// ---------------------------------------------------------------------------
// Canonical group sums for the fused small merges.  Term j of a sweep (a
// pole, or a root for the Loewner products) belongs to partial s = j mod 16,
// which accumulates its terms in increasing j; the 16 partials meet in one
// fixed tree: s with 15 - s, then s with 7 - s within each half, then s with
// s ^ 2, then s with s ^ 1.  A group of G lanes (G = 4, 8 or 16) gives lane l
// the 16 / G partials that the first log2(16 / G) tree steps fold onto l
// (G = 16: l; 8: l, 15 - l; 4: l, 15 - l, 7 - l, 8 + l), folds them locally in
// tree order and takes the remaining steps as DPP lane moves.  Every G gives
// the same bits, so the lanes per root can follow the level's parallelism
// (many lanes per root when a level has few merges, few when it has many)
// without changing any result: a batched solve still equals the single ones.
// ---------------------------------------------------------------------------
template <int G>
struct Canon {
    static_assert(G == 4 || G == 8 || G == 16, "canonical groups of 4, 8 or 16 lanes");
    static constexpr int M = 16 / G;  // partials per lane
    __device__ __forceinline__ static int slot(int l, int q) {
        return q == 0 ? l : (q == 1 ? 15 - l : (q == 2 ? 7 - l : 8 + l));
    }
    __device__ __forceinline__ static double fold_sum(const double* p) {
        if (M == 1) return p[0];
        if (M == 2) return p[0] + p[1];
        return (p[0] + p[1]) + (p[2] + p[3]);
    }
    __device__ __forceinline__ static double fold_prod(const double* p) {
        if (M == 1) return p[0];
        if (M == 2) return p[0] * p[1];
        return (p[0] * p[1]) * (p[2] * p[3]);
    }
    __device__ __forceinline__ static double sum(const double* p) {
        double x = fold_sum(p);
        if (G >= 16) x += dpp_move<kDppMirror>(x);
        if (G >= 8) x += dpp_move<kDppHalfMirror>(x);
        x += dpp_move<kDppSwap2>(x);
        x += dpp_move<kDppSwap1>(x);
        return x;
    }
    __device__ __forceinline__ static double prod(const double* p) {
        double x = fold_prod(p);
        if (G >= 16) x *= dpp_move<kDppMirror>(x);
        if (G >= 8) x *= dpp_move<kDppHalfMirror>(x);
        x *= dpp_move<kDppSwap2>(x);
        x *= dpp_move<kDppSwap1>(x);
        return x;
    }
};

// Runs body(q, j) for every term j < K of this lane's partials q, in
// increasing j per partial (whole chunks of 16 first, then the tail).
template <int G, class Body>
__device__ __forceinline__ void canon_for(int K, int sub, Body body) {
    constexpr int M = Canon<G>::M;
    int off[M];
#pragma unroll
    for (int q = 0; q < M; ++q) off[q] = Canon<G>::slot(sub, q);
    int c = 0;
    _Pragma("unroll 2") for (; c + 16 <= K; c += 16) {
#pragma unroll
        for (int q = 0; q < M; ++q) body(q, c + off[q]);
    }
#pragma unroll
    for (int q = 0; q < M; ++q)
        if (c + off[q] < K) body(q, c + off[q]);
}

// The same canonical value from one lane: partial(s) accumulates terms
// j = s, s + 16, ... in increasing j; the partials meet in the tree above:
// B_q = (P_q + P_15-q) + (P_7-q + P_8+q) for q < 4, then (B_0 + B_2) +
// (B_1 + B_3).  The B_q are formed one per loop trip (in the order 0, 2, 1,
// 3) so that only four partials are live at a time.  Addition and
// multiplication commute exactly, so the order inside each pair is free.
template <class Part, class Op>
__device__ __forceinline__ auto canon1(Part part, Op op) {
    decltype(part(0)) c0{}, c1{};
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        const int q = (t == 0) ? 0 : ((t == 1) ? 2 : ((t == 2) ? 1 : 3));
        const auto b = op(op(part(q), part(15 - q)), op(part(7 - q), part(8 + q)));
        if (t == 0) c0 = b;
        else if (t == 1) c0 = op(c0, b);
        else if (t == 2) c1 = b;
        else c1 = op(c1, b);
    }
    return op(c0, c1);
}

struct Sums4 {
    double a, b, c, d;
};
__device__ __forceinline__ Sums4 add4(const Sums4& x, const Sums4& y) {
    return Sums4{x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d};
}
struct Sums3 {
    double a, b, c;
};
__device__ __forceinline__ Sums3 add3(const Sums3& x, const Sums3& y) { return Sums3{x.a + y.a, x.b + y.b, x.c + y.c}; }
__device__ __forceinline__ double add1(double x, double y) { return x + y; }
__device__ __forceinline__ double mul1(double x, double y) { return x * y; }

// sec_sweep with canonical partial sums (same per-term arithmetic): a group of
// G = 4, 8 or 16 lanes, or one lane (G = 1).
template <int G, bool ZZ>
__device__ __forceinline__ void sec_sweep_c(int K, const double* __restrict__ D, const double* __restrict__ W,
                                            double Do, double tau, int L1, int R0, int sub, double* s) {
    if constexpr (G == 1) {
        static_assert(!ZZ, "one-lane sweeps sum z^2 separately");
        const unsigned exw = (unsigned)(R0 - L1);
        const Sums4 r = canon1(
            [&](int q) {
                Sums4 a{0.0, 0.0, 0.0, 0.0};
                for (int j = q; j < K; j += 16) {
                    const double wr = W[j];
                    const double rr = rcp_nr((D[j] - Do) - tau);
                    const double wj = ((unsigned)(j - L1) < exw) ? 0.0 : wr;
                    const double t = wj * rr;
                    const double tl = fmin(t, 0.0), th = fmax(t, 0.0);
                    a.a += tl;
                    a.b = fma(tl, rr, a.b);
                    a.c += th;
                    a.d = fma(th, rr, a.d);
                }
                return a;
            },
            add4);
        s[0] = r.a;
        s[1] = r.b;
        s[2] = r.c;
        s[3] = r.d;
    } else {
        constexpr int M = Canon<G>::M;
        double ps[M], dps[M], ph[M], dph[M], zz[M];
#pragma unroll
        for (int q = 0; q < M; ++q) ps[q] = dps[q] = ph[q] = dph[q] = zz[q] = 0.0;
        const unsigned exw = (unsigned)(R0 - L1);
        canon_for<G>(K, sub, [&](int q, int j) {
            const double wr = W[j];
            const double rr = rcp_nr((D[j] - Do) - tau);
            const double wj = ((unsigned)(j - L1) < exw) ? 0.0 : wr;
            const double t = wj * rr;
            const double tl = fmin(t, 0.0), th = fmax(t, 0.0);
            ps[q] += tl;
            dps[q] = fma(tl, rr, dps[q]);
            ph[q] += th;
            dph[q] = fma(th, rr, dph[q]);
            if (ZZ) zz[q] += wr;
        });
        s[0] = Canon<G>::sum(ps);
        s[1] = Canon<G>::sum(dps);
        s[2] = Canon<G>::sum(ph);
        s[3] = Canon<G>::sum(dph);
        if (ZZ) s[4] = Canon<G>::sum(zz);
    }
}

// Canonical sum of W[0..K).
template <int G>
__device__ __forceinline__ double canon_wsum(int K, const double* __restrict__ W, int sub) {
    if constexpr (G == 1) {
        return canon1(
            [&](int q) {
                double a = 0.0;
                for (int j = q; j < K; j += 16) a += W[j];
                return a;
            },
            add1);
    } else {
        constexpr int M = Canon<G>::M;
        double zz[M];
#pragma unroll
        for (int q = 0; q < M; ++q) zz[q] = 0.0;
        canon_for<G>(K, sub, [&](int q, int j) { zz[q] += W[j]; });
        return Canon<G>::sum(zz);
    }
}


// secular_root with canonical sweeps (same iteration and stopping rules).
template <int G>
__device__ __forceinline__ int secular_root_c(int k, int K, const double* __restrict__ D,
                                              const double* __restrict__ Z, const double* __restrict__ W, double rho,
                                              int sub, int cap, int* org_out, double* tau_out) {
    if (K == 1) {
        *org_out = 0;
        *tau_out = rho * Z[0] * Z[0];
        return 0;
    }
    const int kk = (k < K - 1) ? k : K - 2;
    SecRoot r;
    double s[5];
    if (k < K - 1) {
        sec_sweep_c<G, false>(K, D, W, D[kk], 0.5 * (D[kk + 1] - D[kk]), kk, kk + 2, sub, s);
        if (sec_start_interior(k, D, Z, rho, s[0], s[1], s[2], s[3], &r)) {
            *org_out = r.o;
            *tau_out = r.tau;
            return 0;
        }
    } else {
        sec_start_last(K, D, Z, rho, canon_wsum<G>(K, W, sub), &r);
    }
    for (int it = 1; it <= cap; ++it) {
        int L1, R0;
        sec_split(r, kk, &L1, &R0);
        sec_sweep_c<G, false>(K, D, W, D[r.o], r.tau, L1, R0, sub, s);
        if (sec_update(&r, rho, s[0], s[1], s[2], s[3], s[2] - s[0])) {
            *org_out = r.o;
            *tau_out = r.tau;
            return it;
        }
    }
    *org_out = r.o;
    *tau_out = r.tau;
    return -1;
}

// lowner_z with canonical partial products: each partial multiplies its
// factors 8 at a time (one division per 8 of its factors), as lowner_z does.
template <int G>
__device__ __forceinline__ double lowner_z_c(int i, int K, const double* __restrict__ D,
                                             const double* __restrict__ Z, const int* __restrict__ org,
                                             const double* __restrict__ tau, double rho, int sub) {
    const double di = D[i];
    if constexpr (G == 1) {
        const double z2 = canon1(
                              [&](int q) {
                                  double prod = 1.0, pn = 1.0, pd = 1.0;
                                  int cnt = 0;
                                  for (int k = q; k < K; k += 16) {
                                      const double num = (D[org[k]] - di) + tau[k];
                                      double den;
                                      if (k < i) den = D[k] - di;
                                      else if (k < K - 1) den = D[k + 1] - di;
                                      else den = 1.0;
                                      pn *= num;
                                      pd *= den;
                                      if (++cnt == 8) {
                                          prod *= pn / pd;
                                          pn = 1.0;
                                          pd = 1.0;
                                          cnt = 0;
                                      }
                                  }
                                  return prod * (pn / pd);
                              },
                              mul1) /
                          rho;
        const double zi = sqrt(fmax(z2, 0.0));
        return (Z[i] < 0.0) ? -zi : zi;
    } else {
        constexpr int M = Canon<G>::M;
        double prod[M], pn[M], pd[M];
        int cnt[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            prod[q] = pn[q] = pd[q] = 1.0;
            cnt[q] = 0;
        }
        canon_for<G>(K, sub, [&](int q, int k) {
            const double num = (D[org[k]] - di) + tau[k];
            double den;
            if (k < i) den = D[k] - di;
            else if (k < K - 1) den = D[k + 1] - di;
            else den = 1.0;
            pn[q] *= num;
            pd[q] *= den;
            if (++cnt[q] == 8) {
                prod[q] *= pn[q] / pd[q];
                pn[q] = 1.0;
                pd[q] = 1.0;
                cnt[q] = 0;
            }
        });
#pragma unroll
        for (int q = 0; q < M; ++q) prod[q] *= pn[q] / pd[q];
        const double z2 = Canon<G>::prod(prod) / rho;
        const double zi = sqrt(fmax(z2, 0.0));
        return (Z[i] < 0.0) ? -zi : zi;
    }
}

// root_rows with canonical partial sums.
template <int G>
__device__ __forceinline__ void root_rows_c(int K, const double* __restrict__ D, const double* __restrict__ zh,
                                            const double* __restrict__ RL, const double* __restrict__ RH, int org,
                                            double tau, int sub, double* bl_out, double* bh_out) {
    const double Do = D[org];
    if constexpr (G == 1) {
        const Sums3 r = canon1(
            [&](int q) {
                Sums3 a{0.0, 0.0, 0.0};
                for (int i = q; i < K; i += 16) {
                    const double y = zh[i] * rcp_nr((D[i] - Do) - tau);
                    a.a = fma(y, y, a.a);
                    a.b = fma(RL[i], y, a.b);
                    a.c = fma(RH[i], y, a.c);
                }
                return a;
            },
            add3);
        const double inv = 1.0 / sqrt(r.a);
        *bl_out = r.b * inv;
        *bh_out = r.c * inv;
    } else {
        constexpr int M = Canon<G>::M;
        double ss[M], bl[M], bh[M];
#pragma unroll
        for (int q = 0; q < M; ++q) ss[q] = bl[q] = bh[q] = 0.0;
        canon_for<G>(K, sub, [&](int q, int i) {
            const double y = zh[i] * rcp_nr((D[i] - Do) - tau);
            ss[q] = fma(y, y, ss[q]);
            bl[q] = fma(RL[i], y, bl[q]);
            bh[q] = fma(RH[i], y, bh[q]);
        });
        const double inv = 1.0 / sqrt(Canon<G>::sum(ss));
        *bl_out = Canon<G>::sum(bl) * inv;
        *bh_out = Canon<G>::sum(bh) * inv;
    }
}

// The root steps of an in-wave level (k_level_wave): G lanes per active root
// (64 / G roots at a time), each merge's arrays read in place from the level
// arrays in LDS; the same arithmetic and canonical sums as small_merge_body.
template <int G>
__device__ void wave_roots_canon(const MergeRec* smr, int K, const double* __restrict__ e,
                                 const unsigned long long* __restrict__ pmax, const Work& wl,
                                 int* __restrict__ corg, double* __restrict__ ctau, long long pk0, WaveCount& c) {
    const int lane = threadIdx.x & 63;
    const int sub = lane % G;
    for (int g = lane / G; g < K; g += 64 / G) {  // group-uniform
        const MergeRec R = smr[wl.amerge[g]];
        const MergeSpan sp = merge_span(R, wl.scan);
        double sgn;
        const double rho = merge_rho(R, e, pmax, &sgn);
        const double* D = wl.Da + sp.ks;
        int o;
        double tau;
        const int it = secular_root_c<G>((int)(g - sp.ks), sp.K, D, wl.Za + sp.ks, wl.Wa + sp.ks, rho, sub,
                                         wl.sec_cap, &o, &tau);
        if (sub == 0) {
            if (it < 0) c.bad = 1;
            wl.org[g] = o;
            wl.tau[g] = tau;
            wl.rootval[g] = D[o] + tau;
            const unsigned long long sw = (sp.K > 1) ? (unsigned long long)((it < 0 ? wl.sec_cap : it) + 1) : 0ULL;
            c.sweeps += sw;
            c.terms += sw * (unsigned long long)sp.K;
            c.roots += 1;
            if (corg) {
                const long long gp = pk0 + R.pk + (g - sp.ks);
                corg[gp] = o;
                ctau[gp] = tau;
            }
        }
    }
    __syncthreads();
    for (int g = lane / G; g < K; g += 64 / G) {
        const MergeRec R = smr[wl.amerge[g]];
        if ((R.flags & MF_ROOT) && !wl.rows_out) continue;  // group-uniform
        const MergeSpan sp = merge_span(R, wl.scan);
        double sgn;
        const double rho = merge_rho(R, e, pmax, &sgn);
        const double zh = lowner_z_c<G>((int)(g - sp.ks), sp.K, wl.Da + sp.ks, wl.Za + sp.ks, wl.org + sp.ks,
                                        wl.tau + sp.ks, rho, sub);
        if (sub == 0) {
            wl.zhat[g] = zh;
            c.lpairs += (unsigned long long)sp.K;
        }
    }
    __syncthreads();
    for (int g = lane / G; g < K; g += 64 / G) {
        const MergeRec R = smr[wl.amerge[g]];
        if ((R.flags & MF_ROOT) && !wl.rows_out) continue;
        const MergeSpan sp = merge_span(R, wl.scan);
        double bl, bh;
        root_rows_c<G>(sp.K, wl.Da + sp.ks, wl.zhat + sp.ks, wl.RLa + sp.ks, wl.RHa + sp.ks, wl.org[g], wl.tau[g],
                       sub, &bl, &bh);
        if (sub == 0) {
            wl.PBL[g] = bl;
            wl.PBH[g] = bh;
            c.rpairs += (unsigned long long)sp.K;
        }
    }
    __syncthreads();
}

// cbase: the first of the four counters (terms, Loewner pairs, row pairs,
// roots) that single out this kernel's share of the work.
template <int NT, int G>
__device__ __forceinline__ void small_merge_body(const MergeRec& R, int K, long long ks, double rho, const Work& w,
                                                 double* sD, double* sW, double* sZ, double* sT, double* sH,
                                                 double* sL, double* sR, int* sO, int cbase) {
    const int sub = threadIdx.x % G, grp = threadIdx.x / G, ng = NT / G;
    int bad = 0;
    unsigned long long terms = 0, sweeps = 0, roots = 0, pairs = 0;
    for (int k = grp; k < K; k += ng) {
        int o;
        double tau;
        const int it = secular_root_c<G>(k, K, sD, sZ, sW, rho, sub, w.sec_cap, &o, &tau);
        if (it < 0) bad = 1;
        if (sub == 0) {
            sO[k] = o;
            sT[k] = tau;
            const unsigned long long sw = (K > 1) ? (unsigned long long)((it < 0 ? w.sec_cap : it) + 1) : 0ULL;
            sweeps += sw;
            terms += sw * (unsigned long long)K;
            roots += 1;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < K; i += NT) {
        w.org[ks + i] = sO[i];
        w.tau[ks + i] = sT[i];
        w.rootval[ks + i] = sD[sO[i]] + sT[i];
    }
    if (!(R.flags & MF_ROOT) || w.rows_out) {
        for (int i = grp; i < K; i += ng) {
            const double zh = lowner_z_c<G>(i, K, sD, sZ, sO, sT, rho, sub);
            if (sub == 0) {
                sH[i] = zh;
                w.zhat[ks + i] = zh;
                pairs += (unsigned long long)K;
            }
        }
        __syncthreads();
        for (int k = grp; k < K; k += ng) {
            double bl, bh;
            root_rows_c<G>(K, sD, sH, sL, sR, sO[k], sT[k], sub, &bl, &bh);
            if (sub == 0) {
                w.PBL[ks + k] = bl;
                w.PBH[ks + k] = bh;
            }
        }
    }
    if (bad && sub == 0) atomicOr(w.status, ST_SEC_NOCONV);
    count_add(w.counters, CNT_SEC_TERMS, terms);
    count_add(w.counters, CNT_SWEEPS, sweeps);
    count_add(w.counters, CNT_ROOTS, roots);
    count_add(w.counters, CNT_LOW_PAIRS, pairs);
    count_add(w.counters, CNT_ROW_PAIRS, pairs);
    count_add(w.counters, cbase, terms);
    count_add(w.counters, cbase + 1, pairs);
    count_add(w.counters, cbase + 2, pairs);
    count_add(w.counters, cbase + 3, roots);
}

// LDS staging of one merge's active arrays for the fused root steps (room
// for CAP active columns).
template <int CAP>
struct SmallStageT {
    double D[CAP], W[CAP], Z[CAP], T[CAP], H[CAP], L[CAP], R[CAP];
    int O[CAP];
};
using SmallStage = SmallStageT<kFuseMax>;

// Roots, Loewner z and rows of one merge with 1 <= K <= CAP active columns at
// active index ks (the whole workgroup; block-uniform arguments).  gmax caps
// the lanes per root (4, 8 or 16); the results do not depend on it.
// With amr (the level's merge table, the merge at index am), the merge's roots
// are then also placed at their parent positions (body_assemble part 1;
// awide: 8-way searches), to aout for a problem's top merge.
template <int NT, class Stage>
__device__ __forceinline__ void small_merge_solve(const MergeRec& R, int K, long long ks, const double* e,
                                                  const unsigned long long* __restrict__ pmax, const Work& w,
                                                  Stage& sg, int cbase, int gmax,
                                                  const MergeRec* __restrict__ amr = nullptr, int am = 0,
                                                  double* __restrict__ aout = nullptr, int awide = 0) {
    for (int i = threadIdx.x; i < K; i += NT) {
        sg.D[i] = w.Da[ks + i];
        sg.W[i] = w.Wa[ks + i];
        sg.Z[i] = w.Za[ks + i];
        sg.L[i] = w.RLa[ks + i];
        sg.R[i] = w.RHa[ks + i];
    }
    double sgn;
    const double rho = merge_rho(R, e, pmax, &sgn);
    __syncthreads();
    // lanes per root: min(16, 1024 / K) rounded down to a power of two, at
    // least 4 (a root's sweeps are latency-bound chains, so on levels of few
    // merges more lanes per root pay even when the workgroup then takes
    // several passes over the roots), capped by gmax (levels of many merges
    // are throughput-bound: fewer lanes per root repeat less of each root's
    // update); the canonical sums make the choice invisible in the results
    const int gk = (K * 16 <= 1024) ? 16 : ((K * 8 <= 1024) ? 8 : 4);
    const int G = gk < gmax ? gk : gmax;
    if (G >= 16) small_merge_body<NT, 16>(R, K, ks, rho, w, sg.D, sg.W, sg.Z, sg.T, sg.H, sg.L, sg.R, sg.O, cbase);
    else if (G >= 8) small_merge_body<NT, 8>(R, K, ks, rho, w, sg.D, sg.W, sg.Z, sg.T, sg.H, sg.L, sg.R, sg.O, cbase);
    else small_merge_body<NT, 4>(R, K, ks, rho, w, sg.D, sg.W, sg.Z, sg.T, sg.H, sg.L, sg.R, sg.O, cbase);
    if (amr != nullptr) {  // block-uniform
        __syncthreads();    // every root's value and rows are stored
        for (int k = threadIdx.x; k < K; k += NT) {
            if (awide) body_assemble<true>(R.pk + k, am, amr, pmax, w, aout, 1);
            else body_assemble<false>(R.pk + k, am, amr, pmax, w, aout, 1);
        }
    }
}

template <int NT>
__device__ void small_merge_fold(int m, const MergeRec* __restrict__ mr, const double* __restrict__ e,
                                 const unsigned long long* __restrict__ pmax, const Work& w, int gmax, int fuse_max,
                                 double* stage, double* out, int amode) {
    const MergeRec R = mr[m];
    const MergeSpan sp = merge_span(R, w.scan);
    const int K = sp.K;
    if (K < 1 || K > fuse_max || K > kFoldCap) return;  // block-uniform
    static_assert(sizeof(SmallStageT<kFoldCap>) <= 2 * kStage * sizeof(double), "stage fits the tiles' LDS");
    SmallStageT<kFoldCap>& sg = *reinterpret_cast<SmallStageT<kFoldCap>*>(stage);
    small_merge_solve<NT>(R, K, sp.ks, e, pmax, w, sg, CNT_SM_TERMS, gmax, amode ? mr : nullptr, m, out, amode == 2);
}

// One workgroup of NT threads per merge of the level; CAP >= the level's
// largest merge (so >= every K), staged in LDS.
template <int NT, int CAP>
__global__ __launch_bounds__(NT) void k_small_merge(const MergeRec* __restrict__ mr, const double* __restrict__ e,
                                                    const unsigned long long* __restrict__ pmax, Work w, int gmax,
                                                    int fuse_max, double* __restrict__ out, int amode) {
    if (input_nonfinite(w)) return;
    const MergeRec R = mr[blockIdx.x];
    const MergeSpan sp = merge_span(R, w.scan);
    const int K = sp.K;
    if (K < 1 || K > fuse_max || K > CAP) return;  // block-uniform
    __shared__ SmallStageT<CAP> sg;
    small_merge_solve<NT>(R, K, sp.ks, e, pmax, w, sg, CNT_SM_TERMS, gmax, amode ? mr : nullptr, (int)blockIdx.x, out,
                          amode == 2);
}

// ---------------------------------------------------------------------------
// Levels whose merges all have at most kFuseMax columns (outside checkpoint
// mode): one workgroup per merge runs the whole merge -- merged order and z~,
// negligible-z flags, close-pole runs, the three-way split, roots, Loewner z,
// rows and the assembly -- with barriers between the steps instead of kernel
// boundaries and merge-local prefix counts instead of level-wide scans: one
// launch per level instead of six.  The per-column and per-root device
// functions are those of the level-wide kernels; they see the merge's active
// and rotated lists and its candidate list through views that start at the
// merge's packed position pk (a merge's lists never outgrow its own range),
// while the negligible list is indexed by pk itself, as body_assemble reads it
// with local counts.  The prefix arrays are shifted by one slot per merge so
// that neighbouring merges' counts (s + 1 entries each) do not overlap.
// ---------------------------------------------------------------------------
// Above this many merges a level keeps the level-wide kernels: they stream the
// columns with all lanes busy, while a workgroup per merge would queue
// thousands of mostly idle 512-thread groups (a merge's result is the same
// either way).
// Levels of merges of at most kLevelBlockSmallCols columns always take them:
// their workgroups are sized to the merge (64 or 128 threads, a few KB of
// LDS), so even tens of thousands of them do not crowd the compute units.
constexpr int kLevelBlockMaxMerges = 1024;
#ifndef TDE_LEVEL_BLOCK_SMALL_COLS
#define TDE_LEVEL_BLOCK_SMALL_COLS 128
#endif
constexpr int kLevelBlockSmallCols = TDE_LEVEL_BLOCK_SMALL_COLS;

// Levels of more merges than this, all of at most kDcCols columns, run in
// waves (k_level_wave) in the forward passes that keep no rows; fewer merges
// keep k_level_block, whose wider workgroups shorten each merge's chain.
#ifndef TDE_LEVEL_WAVE_MIN_MERGES
#define TDE_LEVEL_WAVE_MIN_MERGES 1024
#endif
constexpr int kLevelWaveMinMerges = TDE_LEVEL_WAVE_MIN_MERGES;

static bool level_waved(const LevelInfo& L) { return L.nwp > 0 && L.M > kLevelWaveMinMerges; }

// Levels run by k_level_block or k_level_wave (forward; the reverse pass reads
// their checkpointed roots from the merges' packed positions).
static bool level_blocked(const LevelInfo& L) {
    return level_waved(L) || (L.smax <= kFuseMax && (L.M <= kLevelBlockMaxMerges || L.smax <= kLevelBlockSmallCols));
}

template <int NT, int CAP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_level_block(
    const MergeRec* __restrict__ mr, const double* __restrict__ e,
                                                    const unsigned long long* __restrict__ pmax, Work w,
                                                    double* __restrict__ out, int gmax) {
    if (input_nonfinite(w)) return;
    __shared__ MergeRec sm[1];
    __shared__ int wsum[16];
    __shared__ SmallStageT<CAP> sg;
    const MergeRec R = mr[blockIdx.x];
    if (threadIdx.x == 0) sm[0] = R;
    const int s = R.nL + R.nR;
    const long long pk = R.pk;
    Work v = w;
    // merge b's counts live at [pk + b, pk + b + s]: its total (index pk + s of
    // the view) must not land on the next merge's first count
    v.scan = w.scan + blockIdx.x;
    v.scanC = w.scanC + blockIdx.x;
    v.scanR = w.scanR + blockIdx.x;
    v.nnpos = w.nnpos + pk;
    v.Da = w.Da + pk;
    v.Za = w.Za + pk;
    v.Wa = w.Wa + pk;
    v.RLa = w.RLa + pk;
    v.RHa = w.RHa + pk;
    v.org = w.org + pk;
    v.tau = w.tau + pk;
    v.rootval = w.rootval + pk;
    v.zhat = w.zhat + pk;
    v.PBL = w.PBL + pk;
    v.PBH = w.PBH + pk;
    v.Dr = w.Dr + pk;
    v.RLr = w.RLr + pk;
    v.RHr = w.RHr + pk;
    __syncthreads();
    // merged order, z~, negligible-z flags
    for (int i = threadIdx.x; i < s; i += NT) {
        int f;
        body_merge(pk + i, 0, sm, e, pmax, v, &f);
    }
    __syncthreads();
    // candidates: merge-local prefix counts and positions (each thread a run
    // of consecutive columns)
    const int cs = (s + NT - 1) / NT;
    const int c0 = min(s, (int)threadIdx.x * cs), c1 = min(s, c0 + cs);
    int cnt = 0;
    for (int i = c0; i < c1; ++i) cnt += (v.st[pk + i] == 1) ? 1 : 0;
    const int incl = block_incl_scan(cnt, wsum);
    int g = incl - cnt;
    for (int i = c0; i < c1; ++i) {
        v.scanC[pk + i] = g;
        if (v.st[pk + i] == 1) v.nnpos[g++] = (int)(pk + i);
    }
    if (threadIdx.x == NT - 1) v.scanC[pk + s] = incl;
    __syncthreads();
    // close-pole runs
    const int nc = v.scanC[pk + s];
    for (int q = threadIdx.x; q < nc; q += NT) body_runs(q, 0, sm, v, [](long long) {});
    __syncthreads();
    // three-way split
    int ca = 0, cr = 0;
    for (int i = c0; i < c1; ++i) {
        const int st = v.st[pk + i];
        ca += (st == 1) ? 1 : 0;
        cr += (st == 2) ? 1 : 0;
    }
    const int ia = block_incl_scan(ca, wsum);
    __syncthreads();
    const int ir = block_incl_scan(cr, wsum);
    int ga = ia - ca, gr = ir - cr;
    for (int i = c0; i < c1; ++i) {
        const long long t = pk + i;
        const int st = v.st[t];
        v.scan[t] = ga;
        v.scanR[t] = gr;
        if (st == 1) {
            const double z = v.Z2[t];
            v.Da[ga] = v.D2[t];
            v.Za[ga] = z;
            v.Wa[ga] = z * z;
            v.RLa[ga] = v.RL2[t];
            v.RHa[ga] = v.RH2[t];
            ++ga;
        } else if (st == 2) {
            v.Dr[gr] = v.D2[t];
            v.RLr[gr] = v.RL2[t];
            v.RHr[gr] = v.RH2[t];
            ++gr;
        } else {
            const long long q = pk + (i - ga - gr);
            v.Dd[q] = v.D[t];
            v.RLd[q] = v.RL[t];
            v.RHd[q] = v.RH[t];
        }
    }
    if (threadIdx.x == NT - 1) {
        v.scan[pk + s] = ia;
        v.scanR[pk + s] = ir;
    }
    __syncthreads();
    // roots, Loewner z, rows
    const int K = v.scan[pk + s];
    if (K >= 1) small_merge_solve<NT>(R, K, 0, e, pmax, v, sg, CNT_LB_TERMS, gmax);
    __syncthreads();
    // the parent's spectrum and rows, or the problem's eigenvalues
    for (int i = threadIdx.x; i < s; i += NT) body_assemble(pk + i, 0, sm, pmax, v, out);
    if (threadIdx.x == 0) count_add1(w.counters, CNT_MERGE_COLS, (unsigned long long)s);
}

template <int G, bool WithRoot>
__global__ __launch_bounds__(kWG) void k_lowner(const MergeRec* __restrict__ mr, int M, long long N,
                                                const double* __restrict__ e,
                                                const unsigned long long* __restrict__ pmax, Work w, int wide_min,
                                                int fuse_max, int nbn, const int* __restrict__ blkm, Grad gr,
                                                int nbu, int wsearch, double* __restrict__ out) {
    if (input_nonfinite(w)) return;
    __shared__ double smem[2 * kStage];
    __shared__ int sO[kStage];
    __shared__ long long s_r0;
    __shared__ int s_staged;
    // the last nbu workgroups: in the reverse pass they gather the parent's
    // adjoints onto the level's three lists, in the forward pass they place
    // the deflated columns at their parent positions (body_assemble part 2;
    // the roots are placed by the kernels that finish them); neither needs
    // z-hat, so both share its launch
    const int nbl = (int)gridDim.x - nbu;
    if ((int)blockIdx.x >= nbl) {
        const long long t = ((long long)blockIdx.x - nbl) * kWG + threadIdx.x;
        if (t < N) {
            const int m = merge_of(mr, blkm, t);
            if (WithRoot) {
                if (wsearch) body_bwd_unassemble<true>(t, m, mr, w, gr);
                else body_bwd_unassemble<false>(t, m, mr, w, gr);
            } else {
                if (wsearch) body_assemble<true>(t, m, mr, pmax, w, out, 2);
                else body_assemble<false>(t, m, mr, pmax, w, out, 2);
            }
        }
        return;
    }
    if ((int)blockIdx.x >= nbn) {
        const int* items = w.witems;
        lowner_wide<kWideWaves, false>((int)blockIdx.x - nbn, nbl - nbn, mr, M, e, pmax, w, WithRoot, items, smem);
        return;
    }
    double* sD = smem;
    double* sT = smem + kStage;
    const long long total = min((long long)w.scan[N], N);
    const int per = kWG / G;
    const int sub = threadIdx.x % G;
    unsigned long long pairs = 0;
    for (long long tile = blockIdx.x; tile * per < total; tile += nbn) {
        const long long g0 = tile * per;
        const long long g1 = (g0 + per < total ? g0 + per : total) - 1;
        if (threadIdx.x == 0) {
            const TileWindow tw = tile_window(g0, g1, mr, w, kStage);
            s_r0 = tw.r0;
            s_staged = tw.staged ? (int)(tw.r1 - tw.r0) : -1;
        }
        __syncthreads();
        const long long r0 = s_r0;
        const int ns = s_staged;
        if (ns >= 0)
            for (int i = threadIdx.x; i < ns; i += kWG) {
                sD[i] = w.Da[r0 + i];
                sT[i] = w.tau[r0 + i];
                sO[i] = w.org[r0 + i];
            }
        __syncthreads();
        const long long g = g0 + threadIdx.x / G;
        const int Kg = (g < total) ? merge_span(mr[w.amerge[g]], w.scan).K : 0;
        if (g < total && Kg < wide_min && Kg > fuse_max) {
            const int m = w.amerge[g];
            if (ns >= 0) body_lowner<RedGroup<G>>(g, m, mr, e, pmax, w, sub, G, sD, sO, sT, r0, WithRoot);
            else body_lowner<RedGroup<G>>(g, m, mr, e, pmax, w, sub, G, w.Da, w.org, w.tau, 0, WithRoot);
            if (sub == 0 && (!(mr[m].flags & MF_ROOT) || w.rows_out)) pairs += (unsigned long long)merge_span(mr[m], w.scan).K;
        }
        __syncthreads();
    }
    count_add(w.counters, CNT_LOW_PAIRS, pairs);
}

// amode 1 or 2 (no wide blocks then): each root is also placed at its parent
// position by the lane that stored its rows (body_assemble part 1; 2: 8-way
// searches), to out for a problem's top merge.
template <int G>
__global__ __launch_bounds__(kWG) void k_rows(const MergeRec* __restrict__ mr, int M, long long N, Work w,
                                              int wide_min, int fuse_max, int nbn,
                                              const unsigned long long* __restrict__ pmax, double* __restrict__ out,
                                              int amode) {
    if (input_nonfinite(w)) return;
    __shared__ double smem[4 * kStageRows];
    __shared__ long long s_r0;
    __shared__ int s_staged;
    if ((int)blockIdx.x >= nbn) {
        const int* items = w.witems;
        rows_wide<kWideWaves>((int)blockIdx.x - nbn, (int)gridDim.x - nbn, mr, M, w, items, smem);
        return;
    }
    double* sD = smem;
    double* sH = smem + kStageRows;
    double* sL = smem + 2 * kStageRows;
    double* sR = smem + 3 * kStageRows;
    const long long total = min((long long)w.scan[N], N);
    const int per = kWG / G;
    const int sub = threadIdx.x % G;
    unsigned long long pairs = 0;
    for (long long tile = blockIdx.x; tile * per < total; tile += nbn) {
        const long long g0 = tile * per;
        const long long g1 = (g0 + per < total ? g0 + per : total) - 1;
        if (threadIdx.x == 0) {
            const TileWindow tw = tile_window(g0, g1, mr, w, kStageRows);
            s_r0 = tw.r0;
            s_staged = tw.staged ? (int)(tw.r1 - tw.r0) : -1;
        }
        __syncthreads();
        const long long r0 = s_r0;
        const int ns = s_staged;
        if (ns >= 0)
            for (int i = threadIdx.x; i < ns; i += kWG) {
                sD[i] = w.Da[r0 + i];
                sH[i] = w.zhat[r0 + i];
                sL[i] = w.RLa[r0 + i];
                sR[i] = w.RHa[r0 + i];
            }
        __syncthreads();
        const long long g = g0 + threadIdx.x / G;
        const int Kg = (g < total) ? merge_span(mr[w.amerge[g]], w.scan).K : 0;
        if (g < total && Kg < wide_min && Kg > fuse_max) {
            const int m = w.amerge[g];
            if (ns >= 0) body_rows<RedGroup<G>>(g, m, mr, w, sub, G, sD, sH, sL, sR, r0);
            else body_rows<RedGroup<G>>(g, m, mr, w, sub, G, w.Da, w.zhat, w.RLa, w.RHa, 0);
            if (sub == 0 && (!(mr[m].flags & MF_ROOT) || w.rows_out)) pairs += (unsigned long long)merge_span(mr[m], w.scan).K;
            if (amode && sub == 0) {
                const long long t = mr[m].pk + (g - merge_span(mr[m], w.scan).ks);
                if (amode == 2) body_assemble<true>(t, m, mr, pmax, w, out, 1);
                else body_assemble<false>(t, m, mr, pmax, w, out, 1);
            }
        }
        __syncthreads();
    }
    count_add(w.counters, CNT_ROW_PAIRS, pairs);
}

template <bool Wide>
__global__ __launch_bounds__(kWG) void k_assemble(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                                  long long N, const unsigned long long* __restrict__ pmax, Work w,
                                                  double* __restrict__ out) {
    if (input_nonfinite(w)) return;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < N) body_assemble<Wide>(t, merge_of(mr, blkm, t), mr, pmax, w, out);
}

// ---------------------------------------------------------------------------
// Reverse pass (adjoint).  Level by level from the top, each level first
// recomputes its merged order, deflation and Loewner z from the checkpoint,
// then runs the per-merge VJP steps of tde_adjoint.h; the leaves and the tear
// couplings close the chain.
// ---------------------------------------------------------------------------

// Snapshot of the node spectra and rows the level's merges are about to read.
__global__ __launch_bounds__(kWG) void k_ckpt_save(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                                   long long N, Work w, double* __restrict__ sl,
                                                   double* __restrict__ sb, double* __restrict__ sh) {
    if (input_nonfinite(w)) return;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= N) return;
    const MergeRec R = mr[merge_of(mr, blkm, t)];
    const long long P = R.off + (t - R.pk);
    sl[P] = w.lam[P];
    sb[P] = w.blo[P];
    sh[P] = w.bhi[P];
}

// Seed: dL/dlambda of every output eigenvalue; no row adjoints above the top.
__global__ __launch_bounds__(kWG) void k_bwd_init(long long n, const double* __restrict__ gin, Grad gr) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    gr.glam[t] = gin[t];
    gr.gblo[t] = 0.0;
    gr.gbhi[t] = 0.0;
}

// Roots of a level the forward ran with k_level_block: the checkpoint holds
// them at the merges' packed positions (pk + local index); gather them into
// active-index order for the reverse steps.
__global__ __launch_bounds__(kWG) void k_bwd_roots_gather(const MergeRec* __restrict__ mr, long long N, Work w,
                                                          const int* __restrict__ corg,
                                                          const double* __restrict__ ctau) {
    if (input_nonfinite(w)) return;
    const long long total = min((long long)w.scan[N], N);
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x) {
        const MergeRec R = mr[w.amerge[g]];
        const long long src = R.pk + (g - w.scan[R.pk]);
        w.org[g] = corg[src];
        w.tau[g] = ctau[src];
    }
}


constexpr int kStageBwd = 1024;

template <int G>
__global__ __launch_bounds__(kWG) void k_bwd_roots(const MergeRec* __restrict__ mr, long long N, Work w, Grad gr,
                                                   long long cstride) {
    if (input_nonfinite(w)) return;
    __shared__ double sD[kStageBwd], sH[kStageBwd], sL[kStageBwd], sR[kStageBwd];
    __shared__ long long s_r0;
    __shared__ int s_staged;
    const long long total = min((long long)w.scan[N], N);
    const int per = kWG / G;
    const int sub = threadIdx.x % G;
    for (long long tile = blockIdx.x; tile * per < total; tile += gridDim.x) {
        const long long g0 = tile * per;
        const long long g1 = (g0 + per < total ? g0 + per : total) - 1;
        if (threadIdx.x == 0) {
            const TileWindow tw = tile_window(g0, g1, mr, w, kStageBwd);
            s_r0 = tw.r0;
            s_staged = tw.staged ? (int)(tw.r1 - tw.r0) : -1;
        }
        __syncthreads();
        const long long r0 = s_r0;
        const int ns = s_staged;
        if (ns >= 0)
            for (int i = threadIdx.x; i < ns; i += kWG) {
                sD[i] = w.Da[r0 + i];
                sH[i] = w.zhat[r0 + i];
                sL[i] = w.RLa[r0 + i];
                sR[i] = w.RHa[r0 + i];
            }
        __syncthreads();
        const long long g = g0 + threadIdx.x / G;
        if (g < total) {
            const MergeSpan sp = merge_span(mr[w.amerge[g]], w.scan);
            const long long b = sp.ks - (ns >= 0 ? r0 : 0);
            const double* Dv = (ns >= 0 ? sD : w.Da) + b;
            const double* Hv = (ns >= 0 ? sH : w.zhat) + b;
            const double* Lv = (ns >= 0 ? sL : w.RLa) + b;
            const double* Rv = (ns >= 0 ? sR : w.RHa) + b;
            double cf[10];
            bwd_root_coeffs<RedGroup<G>>(sp.K, Dv, Hv, Lv, Rv, w.org[g], w.tau[g], gr.glr[g], gr.gbr[g], gr.ghr[g],
                                         sub, G, cf);
            if (sub == 0)
                for (int q = 0; q < 10; ++q) gr.coef[q * cstride + g] = cf[q];
        }
        __syncthreads();
    }
}

template <int G>
__global__ __launch_bounds__(kWG) void k_bwd_poles(const MergeRec* __restrict__ mr, long long N, Work w, Grad gr,
                                                   long long cstride) {
    if (input_nonfinite(w)) return;
    __shared__ double sD[kStageBwd], sT[kStageBwd], sA[kStageBwd], sB[kStageBwd], sC[kStageBwd], sM[kStageBwd];
    __shared__ int sO[kStageBwd];
    __shared__ long long s_r0;
    __shared__ int s_staged;
    const long long total = min((long long)w.scan[N], N);
    const int per = kWG / G;
    const int sub = threadIdx.x % G;
    for (long long tile = blockIdx.x; tile * per < total; tile += gridDim.x) {
        const long long g0 = tile * per;
        const long long g1 = (g0 + per < total ? g0 + per : total) - 1;
        if (threadIdx.x == 0) {
            const TileWindow tw = tile_window(g0, g1, mr, w, kStageBwd);
            s_r0 = tw.r0;
            s_staged = tw.staged ? (int)(tw.r1 - tw.r0) : -1;
        }
        __syncthreads();
        const long long r0 = s_r0;
        const int ns = s_staged;
        if (ns >= 0)
            for (int i = threadIdx.x; i < ns; i += kWG) {
                sD[i] = w.Da[r0 + i];
                sT[i] = w.tau[r0 + i];
                sO[i] = w.org[r0 + i];
                sA[i] = gr.coef[r0 + i];
                sB[i] = gr.coef[cstride + r0 + i];
                sC[i] = gr.coef[2 * cstride + r0 + i];
                sM[i] = gr.coef[3 * cstride + r0 + i];
            }
        __syncthreads();
        const long long g = g0 + threadIdx.x / G;
        if (g < total) {
            const MergeSpan sp = merge_span(mr[w.amerge[g]], w.scan);
            const bool stg = ns >= 0;
            const long long b = sp.ks - (stg ? r0 : 0);
            const double* cg = gr.coef + sp.ks;
            double o4[4];
            bwd_pole<RedGroup<G>>((int)(g - sp.ks), sp.K, (stg ? sD : w.Da) + b, (stg ? sO : w.org) + b,
                                  (stg ? sT : w.tau) + b, stg ? sA + b : cg, stg ? sB + b : cg + cstride,
                                  stg ? sC + b : cg + 2 * cstride, stg ? sM + b : cg + 3 * cstride, cg, cstride,
                                  w.zhat[g], w.RLa[g], w.RHa[g], sub, G, o4);
            if (sub == 0) {
                const long long t = w.apos[g];
                gr.gZ2[t] = o4[0];
                gr.gD2[t] = o4[1];
                gr.gRL2[t] = o4[2];
                gr.gRH2[t] = o4[3];
            }
        }
        __syncthreads();
    }
}

// dL/dz of the negligible-z columns of non-top merges: G lanes per column
// (the group splits the sum over the merge's roots).  Groups take the
// level's negligible columns in their compacted order (dpos), so whole
// waves either work or leave.  b: this workgroup's index among those of the
// step.
template <int G>
__device__ __forceinline__ void bwd_negl_block(int b, const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                               long long N, const Work& w, const Grad& gr, long long cstride) {
    const long long q = ((long long)b * blockDim.x + threadIdx.x) / G;
    const int sub = (int)(threadIdx.x % G);
    const long long nneg = N - w.scan[N] - w.scanR[N];
    if (q >= nneg) return;  // group-uniform
    const long long t = w.dpos[q];
    const MergeRec R = mr[merge_of(mr, blkm, t)];
    if (R.flags & MF_ROOT) return;
    const MergeSpan sp = merge_span(R, w.scan);
    const double gz = bwd_negligible_z<RedGroup<G>>(sp.K, w.Da + sp.ks, w.org + sp.ks, w.tau + sp.ks,
                                                    gr.coef + sp.ks, cstride, w.D[t], w.RL[t], w.RH[t], gr.gRL[t],
                                                    gr.gRH[t], sub, G);
    if (sub == 0) gr.gZ[t] = gz;
}

// dL/drho~ of merge m: sum_k gtot_k / (rho^2 N_k^2), one workgroup.
__device__ __forceinline__ void bwd_grho_block(int m, const MergeRec* __restrict__ mr, const double* __restrict__ e,
                                               const unsigned long long* __restrict__ pmax, const Work& w,
                                               const Grad& gr, long long cstride, int mstart, double* part) {
    const MergeRec R = mr[m];
    const MergeSpan sp = merge_span(R, w.scan);
    const double* mu = gr.coef + 3 * cstride + sp.ks;
    double acc = 0.0;
    for (int k = threadIdx.x; k < sp.K; k += kWG) acc += mu[k];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < kWG / 64; ++i) s += part[i];
        double sgn;
        const double rho = merge_rho(R, e, pmax, &sgn);
        gr.grho[mstart + m] = sp.K ? s / (rho * rho) : 0.0;
    }
}

// Candidates one per lane (stride nb workgroups): those in no run pass
// straight through, and each group of G lanes then takes, one after another,
// the runs that start among its G candidates.
template <int G>
__device__ __forceinline__ void bwd_runs_block(int b, int nb, const MergeRec* __restrict__ mr,
                                               const int* __restrict__ blkm, long long N, const Work& w,
                                               const Grad& gr, long long cstride) {
    const long long total = w.scanC[N];
    const int lane = (int)(threadIdx.x & 63);
    const int sub = lane % G;
    const long long stride = (long long)nb * blockDim.x;
    for (long long g0 = (long long)b * blockDim.x + (threadIdx.x - sub); g0 < total; g0 += stride) {
        const long long g = g0 + sub;
        const bool head = g < total && bwd_run_head(g, merge_of(mr, blkm, w.nnpos[g]), mr, w, gr);
        // this group's G bits of the wave's ballot (group-uniform)
        unsigned long long heads = (__ballot(head) >> (lane - sub)) & ((G == 64) ? ~0ull : ((1ull << G) - 1));
        while (heads) {
            const long long h = g0 + __builtin_ctzll(heads);
            heads &= heads - 1;
            body_bwd_runs<RedGroup<G>>(h, merge_of(mr, blkm, w.nnpos[h]), mr, w, gr, cstride, sub, G);
        }
    }
}

// The steps of a level after the pole adjoints, in one launch: workgroups
// [0, nbr) the close-pole runs, [nbr, nbr + nbn) the negligible columns,
// [nbr + nbn, nbr + nbn + M) one merge's dL/drho~ each.  All three read the
// root coefficients and the node's adjoints and write disjoint outputs
// (candidate columns and the runs' scratch, negligible columns, per-merge
// rho), so they need no order among themselves, and the short ones run in
// the long ones' shadow instead of after them.
template <int G>
__global__ __launch_bounds__(kWG) void k_bwd_defl(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                                  long long N, const double* __restrict__ e,
                                                  const unsigned long long* __restrict__ pmax, Work w, Grad gr,
                                                  long long cstride, int mstart, int nbr, int nbn) {
    if (input_nonfinite(w)) return;
    __shared__ double part[kWG / 64];
    const int b = (int)blockIdx.x;
    if (b < nbr) bwd_runs_block<G>(b, nbr, mr, blkm, N, w, gr, cstride);
    else if (b < nbr + nbn) bwd_negl_block<G>(b - nbr, mr, blkm, N, w, gr, cstride);
    else bwd_grho_block(b - nbr - nbn, mr, e, pmax, w, gr, cstride, mstart, part);  // block-uniform
}

__global__ __launch_bounds__(kWG) void k_bwd_merge(const MergeRec* __restrict__ mr, const int* __restrict__ blkm,
                                                   long long N, const double* __restrict__ e,
                                                   const unsigned long long* __restrict__ pmax, Work w, Grad gr) {
    if (input_nonfinite(w)) return;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < N) body_bwd_merge(t, merge_of(mr, blkm, t), mr, e, pmax, w, gr);
}

// Leaves: LMAX / R lanes per leaf, R rows per lane (64 R / LMAX leaves per
// 64-lane workgroup).  Each lane recomputes the QL on its own copy of the leaf
// (LDS, lane-strided) tracking its rows of Q; the leaf's Q (leading dimension
// LMAX) is shared in LDS, and X takes the space of the QL copies once every
// lane is done with them.  Fewer lanes per leaf repeat the QL fewer times.
template <int LMAX, int R>
__global__ __launch_bounds__(64) void k_bwd_leaf(const LeafRec* __restrict__ leaves, int nleaves,
                                                 const double* __restrict__ d, const double* __restrict__ e,
                                                 const unsigned long long* __restrict__ pmax, Work w, Grad gr,
                                                 double* __restrict__ gd, double* __restrict__ ge) {
    if (input_nonfinite(w)) return;
    constexpr int LPL = LMAX / R;  // lanes per leaf
    constexpr int P = 64 / LPL;    // leaves per workgroup
    static_assert(LPL * R == LMAX && P * LPL == 64, "lanes per leaf divide the wave");
    static_assert(P * LMAX * LMAX <= 2 * LMAX * 64, "X fits in the QL copies");
    __shared__ double sde[2 * LMAX * 64];
    __shared__ double sQ[P * LMAX * LMAX], sL[P * LMAX];
    const int lane = threadIdx.x;
    const int slot = lane / LPL, sub = lane % LPL;
    const long long li = (long long)blockIdx.x * P + slot;
    LeafRec L{};
    bool act = false;
    if (li < nleaves) {
        L = leaves[li];
        act = sub < L.size;
    }
    double* Q = sQ + slot * LMAX * LMAX;
    double* lam = sL + slot * LMAX;
    int st = 0;
    if (act) st = bwd_leaf_q<R>(L, sub, LPL, d, e, pmax, sde + lane, sde + LMAX * 64 + lane, 64, Q, LMAX, lam);
    __syncthreads();
    double* X = sde + slot * LMAX * LMAX;
    if (act)
        for (int r = sub; r < L.size; r += LPL) body_bwd_leaf_x(L, r, gr, Q, LMAX, lam, X);
    __syncthreads();
    if (act)
        for (int r = sub; r < L.size; r += LPL) body_bwd_leaf_out(L, r, gr, Q, X, LMAX, gd, ge);
    if (st) atomicOr(w.status, st);
}

__global__ __launch_bounds__(kWG) void k_bwd_tear(const MergeRec* __restrict__ mr, int nm,
                                                  const double* __restrict__ e,
                                                  const unsigned long long* __restrict__ pmax, Grad gr,
                                                  double* __restrict__ ge) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nm) body_bwd_tear(mr[i], gr.grho[i], e, pmax, gr, ge);
}

// The coupling slot after the last row of every problem does not exist: 0.
__global__ __launch_bounds__(kWG) void k_bwd_edges(const long long* __restrict__ offs, int B, double* __restrict__ ge) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B && offs[b + 1] > offs[b]) ge[offs[b + 1] - 1] = 0.0;
}

// Requested rows: sign every eigenvector column like the boundary rows (the
// first entry >= 0, the last when the first is 0; q0 / q1 are the unsigned top
// rows of the same solve) and copy repeated requests from their first
// occurrence.  One thread per column; Q is [m][n], row i at Q + i n.
__global__ __launch_bounds__(kWG) void k_selrows_fix(double* __restrict__ Q, long long m, long long n,
                                                     const int* __restrict__ first, const double* __restrict__ q0,
                                                     const double* __restrict__ q1) {
    const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double a = q0[k], b = q1[k];
    const double sg = (a < 0.0 || (a == 0.0 && b < 0.0)) ? -1.0 : 1.0;
    for (long long i = 0; i < m; ++i)
        if (first[i] == i) Q[i * n + k] *= sg;
    for (long long i = 0; i < m; ++i)
        if (first[i] != i) Q[i * n + k] = Q[(long long)first[i] * n + k];
}

// ---------------------------------------------------------------------------
// Optional per-kernel timing: HIP events recorded on the solve's stream
// around every launch, summed per launch kind on read-back.
// ---------------------------------------------------------------------------
namespace {
struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
thread_local bool t_untimed = false;  // this thread's launches are never timed
std::vector<TimedLaunch> g_timed;

struct TimingScope {
    int kind;
    void* stream;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    TimingScope(int k, void* s) : kind(k), stream(s), on(g_timing && !t_untimed) {
        if (on && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, (hipStream_t)stream);
        else on = false;
    }
    ~TimingScope() {
        if (!on) return;
        if (hipEventCreate(&b) != hipSuccess) return;
        (void)hipEventRecord(b, (hipStream_t)stream);
        std::lock_guard<std::mutex> lk(g_tmu);
        g_timed.push_back(TimedLaunch{kind, a, b});
    }
};
}  // namespace

void timing_enable(bool on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on;
}

void timing_suppress(bool on) { t_untimed = on; }

bool timing_enabled() {
    std::lock_guard<std::mutex> lk(g_tmu);
    return g_timing;
}

int timing_read(double* ms, long long* count, int nkinds) {
    std::vector<TimedLaunch> recs;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        recs.swap(g_timed);
    }
    for (int k = 0; k < nkinds; ++k) {
        ms[k] = 0.0;
        count[k] = 0;
    }
    int rc = 0;
    for (auto& r : recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) rc = -1;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) rc = -1;
        if (r.kind >= 0 && r.kind < nkinds) {
            ms[r.kind] += t;
            count[r.kind] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    return rc;
}

// ---------------------------------------------------------------------------
// Launch sequence
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n, int per) { return (unsigned)((n + per - 1) / per); }

#define TDE_LAUNCH_K(kindv, kern, grid, block, stream, ...)                          \
    do {                                                                             \
        TimingScope ts_((kindv), (stream));                                          \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (hipStream_t)(stream), \
                           __VA_ARGS__);                                             \
    } while (0)
#define TDE_LAUNCH(kern, grid, block, stream, ...) TDE_LAUNCH_K(KIND_DEFLATE, kern, grid, block, stream, __VA_ARGS__)

// Lanes per root: the smallest power of two G <= 16 with G * cols >= smax, so
// that each lane sweeps about `cols` poles of the level's largest merge.
static int lanes_per_root(int smax, int cols) {
    int G = 1;
    while (G < 16 && (long long)G * cols < smax) G <<= 1;
    return G;
}

// Grid of a root kernel: the regular tiles plus, when the level has a merge
// large enough, up to wblocks wide blocks (default kWideGridMax; they loop
// over the level's 64-root items, so a level with more items than blocks
// still gets them all).  The wide launches must be in the graph whenever a
// level has a merge large enough, because the active counts are known only
// on the device; where they find nothing (random spectra), a smaller grid
// costs less, where they carry the solve (Toeplitz-like spectra) a larger
// one keeps more waves per compute unit: the autotuner picks.
constexpr long long kWideGridMax = 4096;
static void root_grid(long long N, int G, bool wide, int* nbn, int* nbw, long long wblocks = kWideGridMax) {
    long long nb = (N * G + kWG - 1) / kWG;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    long long wb = wide ? (N + 63) / 64 : 0;
    if (wb > wblocks) wb = wblocks;
    *nbn = (int)nb;
    *nbw = (int)wb;
}

// Lanes per root of the fused small merges on a level of M merges: a
// caller's cap, else 16 when the level has few merges (latency-bound: every
// lane of a root's group shortens its sweeps) and 4 when it has many
// (throughput-bound: fewer lanes repeat less of each root's update).
constexpr int kFewMerges = 1024;
static int fused_gmax(int M, int group_max) {
    if (group_max > 0) return group_max;
    return M < kFewMerges ? 16 : 4;
}

// Most active roots of a merge that one workgroup solves (k_small_merge) on
// a level of M merges: kFuseMax on levels of many merges (the workgroups fill
// the chip); on levels of few merges the caller's fuse_few when given, so
// that the larger merges go to the root-parallel kernels, which spread a
// merge's roots over many workgroups where a lone workgroup per merge leaves
// most compute units idle.
static int level_fuse_max(int M, int fuse_few) { return (M < kFewMerges && fuse_few > 0) ? fuse_few : kFuseMax; }

// Fused small merges of one level: a workgroup per merge; on levels of many
// merges its shape follows the level's largest merge (LDS room and threads
// for that many active columns), on levels of few it is the full size.
// Assembly searches its three lists 8 ways at a time on levels of at most
// kWideSearchCols columns (few threads, each latency-bound: uniform n = 65536,
// 94 -> 77 us of assembly per solve), binary on larger levels (a batch of
// 4096 problems: the 8-way search was 2% slower there).
constexpr long long kWideSearchCols = 1LL << 18;

static void launch_small(int smax, const MergeRec* mr, int M, const double* e, const Work& w, int gmax, int fuse_max,
                         double* out, int amode, void* stream) {
    const unsigned long long* pm = (const unsigned long long*)w.pmax;
    const unsigned g = (unsigned)M;
    if (smax >= kFuseWideS)
        TDE_LAUNCH_K(KIND_SMALL, (k_small_merge<2 * kFuseThreads, kFuseMax>), g, 2 * kFuseThreads, stream, mr, e, pm,
                     w, gmax, fuse_max, out, amode);
    else if (smax > 256 || M < kFewMerges)
        TDE_LAUNCH_K(KIND_SMALL, (k_small_merge<kFuseThreads, kFuseMax>), g, kFuseThreads, stream, mr, e, pm, w, gmax,
                     fuse_max, out, amode);
    else if (smax > 128)
        TDE_LAUNCH_K(KIND_SMALL, (k_small_merge<256, 256>), g, 256, stream, mr, e, pm, w, gmax, fuse_max, out, amode);
    else if (smax > 64)
        TDE_LAUNCH_K(KIND_SMALL, (k_small_merge<128, 128>), g, 128, stream, mr, e, pm, w, gmax, fuse_max, out, amode);
    else
        TDE_LAUNCH_K(KIND_SMALL, (k_small_merge<128, 64>), g, 128, stream, mr, e, pm, w, gmax, fuse_max, out, amode);
}

// Levels of at most this many merges of more than 128 columns (at most one
// workgroup per compute unit) give each merge 1024 threads: the roots take
// fewer passes (uniform n = 65536: 218 -> 208 us for the three levels;
// Toeplitz: 520 -> 454 us).
constexpr int kLevelBlockWideMerges = 256;

// Whole merges in one workgroup each: 512 threads on other levels of few
// merges (each merge's chain of steps is latency-bound, so more threads per
// merge shorten it), else a workgroup sized to the level's largest merge
// (levels of many merges are throughput-bound).
static void launch_level_block(int smax, const MergeRec* mr, int M, const double* e, const Work& w, double* out,
                               int gmax, void* stream) {
    const unsigned long long* pm = (const unsigned long long*)w.pmax;
    const unsigned g = (unsigned)M;
    if (smax > 128 && M <= kLevelBlockWideMerges)
        TDE_LAUNCH_K(KIND_LEVEL, (k_level_block<2 * kFuseThreads, kFuseMax>), g, 2 * kFuseThreads, stream, mr, e, pm,
                     w, out, gmax);
    else if (smax > 256 || M <= kLevelBlockMaxMerges)
        TDE_LAUNCH_K(KIND_LEVEL, (k_level_block<kFuseThreads, kFuseMax>), g, kFuseThreads, stream, mr, e, pm, w, out,
                     gmax);
    else if (smax > 128)
        TDE_LAUNCH_K(KIND_LEVEL, (k_level_block<256, 256>), g, 256, stream, mr, e, pm, w, out, gmax);
    else if (smax > 64)
        TDE_LAUNCH_K(KIND_LEVEL, (k_level_block<128, 128>), g, 128, stream, mr, e, pm, w, out, gmax);
    else
        TDE_LAUNCH_K(KIND_LEVEL, (k_level_block<64, 64>), g, 64, stream, mr, e, pm, w, out, gmax);
}

// no_rows: every merge of the level is a problem's top merge and no rows
// are requested, so the Loewner and row steps would find nothing to do and
// are not launched.
template <int G>
static bool launch_roots_g(int smax, int wmin, long long N, const MergeRec* mr, const int* blkm, int M,
                           const double* e, const Work& w, double* out, int gmax, int wblocks, int fuse_few,
                           bool no_rows, void* stream) {
    const unsigned long long* pm = (const unsigned long long*)w.pmax;
    const int fuse_max = level_fuse_max(M, fuse_few);
    const bool wide = smax >= wmin;
    const int wide_min = wide ? wmin : 0x7fffffff;
    int nbn, nbw;
    root_grid(N, G, wide, &nbn, &nbw, wblocks);
    // every merge too large for k_small_merge is wide: no regular tiles
    if (wide_min <= fuse_max + 1) nbn = 0;
    // Levels whose roots all come from the fused workgroups and the regular
    // tiles, with row steps: the kernels that finish a root also place it,
    // and the Loewner launch places the deflated columns, so the level needs
    // no assembly launch of its own (the caller is told so).
    const bool placed = !no_rows && smax > fuse_max && nbn > 0 && nbw == 0;
    const int amode = placed ? (N <= kWideSearchCols ? 2 : 1) : 0;
    // merges with at most fuse_max active roots: one workgroup each, inside
    // the tiles' secular launch when there are tiles and those merges are
    // small, else a launch of their own
    const int nsm = (smax > fuse_max && nbn > 0 && fuse_max <= kFoldCap) ? M : 0;
    if (nsm == 0) launch_small(smax, mr, M, e, w, gmax, fuse_max, out, amode, stream);
    if (smax <= fuse_max) return false;  // no merge of the level can have more
    const unsigned grid = (unsigned)(nbn + nbw);
    // one k_wide_items launch serves the three root kernels of the level (on
    // wide-only levels of few merges the secular kernel builds the table)
    const int own_items = (nbn == 0 && M <= kWideOwnItems) ? 1 : 0;
    if (wide && !own_items) TDE_LAUNCH_K(KIND_DEFLATE, k_wide_items, 1, 1024, stream, mr, M, w, wide_min, fuse_max);
    long long rf = (N * G) / kRefillLanes;  // roots per group: keep about kRefillLanes lanes busy
    rf = rf < 1 ? 1 : (rf > kRefillMax ? kRefillMax : rf);
    const int nbs = (int)((nbn + rf - 1) / rf);
    if (nbn == 0) {  // wide blocks only
        const unsigned bw = kWideWavesOnly * 64;
        TDE_LAUNCH_K(KIND_SECULAR, k_secular_wide<kWideWavesOnly>, (unsigned)nbw, bw, stream, mr, M, e, pm, w,
                     wide_min, fuse_max, own_items);
        if (no_rows) return false;
        TDE_LAUNCH_K(KIND_LOWNER, k_lowner_wide<kWideWavesOnly>, (unsigned)nbw, bw, stream, mr, M, e, pm, w);
        TDE_LAUNCH_K(KIND_ROWS, k_rows_wide<kWideWavesOnly>, (unsigned)nbw, bw, stream, mr, M, w);
        return false;
    }
    TDE_LAUNCH_K(KIND_SECULAR, k_secular<G>, (unsigned)(nbs + nbw + nsm), kWG, stream, mr, M, N, e, pm, w, wide_min,
                 fuse_max, nbs, (int)rf, nsm, gmax, out, amode);
    if (no_rows) return false;
    const unsigned nba = placed ? nblk(N, kWG) : 0u;
    TDE_LAUNCH_K(KIND_LOWNER, (k_lowner<G, false>), grid + nba, kWG, stream, mr, M, N, e, pm, w, wide_min, fuse_max,
                 nbn, blkm, Grad{}, (int)nba, N <= kWideSearchCols ? 1 : 0, out);
    TDE_LAUNCH_K(KIND_ROWS, k_rows<G>, grid, kWG, stream, mr, M, N, w, wide_min, fuse_max, nbn, pm, out, amode);
    return placed;
}

// Returns true when the level's columns were placed at their parent
// positions by the root kernels (no assembly launch needed).
static bool launch_roots(int smax, int cols, int wmin, long long N, const MergeRec* mr, const int* blkm, int M,
                         const double* e, const Work& w, double* out, int gmax, int wblocks, int fuse_few,
                         bool no_rows, void* stream) {
    switch (lanes_per_root(smax, cols)) {
        case 1: return launch_roots_g<1>(smax, wmin, N, mr, blkm, M, e, w, out, gmax, wblocks, fuse_few, no_rows, stream);
        case 2: return launch_roots_g<2>(smax, wmin, N, mr, blkm, M, e, w, out, gmax, wblocks, fuse_few, no_rows, stream);
        case 4: return launch_roots_g<4>(smax, wmin, N, mr, blkm, M, e, w, out, gmax, wblocks, fuse_few, no_rows, stream);
        case 8: return launch_roots_g<8>(smax, wmin, N, mr, blkm, M, e, w, out, gmax, wblocks, fuse_few, no_rows, stream);
        default:
            return launch_roots_g<16>(smax, wmin, N, mr, blkm, M, e, w, out, gmax, wblocks, fuse_few, no_rows, stream);
    }
}

// Merged order of one level: by output position (merge path) when the level's
// merges average at least kMergePathMin columns, else one thread per input
// column with its own binary search (few steps for small merges).
constexpr long long kMergePathMin = 1024;
static void launch_merge(int kind, const LevelInfo& L, const MergeRec* mr, const int* blkm, const double* e,
                         const Work& wl, void* stream) {
    const unsigned nb = nblk(L.N, kWG);
    const unsigned long long* pm = (const unsigned long long*)wl.pmax;
    if (L.N >= kMergePathMin * (long long)L.M)
        TDE_LAUNCH_K(kind, k_merge_path, nb, kWG, stream, mr, blkm, L.N, e, pm, wl);
    else
        TDE_LAUNCH_K(kind, k_merge, nb, kWG, stream, mr, blkm, L.N, e, pm, wl);
}

// Deflation steps of one level (shared by the forward and the reverse pass):
// negligible-z flags, candidate compaction, close-pole runs, three-way split.
static void enqueue_deflate(const MergeRec* mr, const int* blkm, long long N, const Work& wl, void* stream) {
    const unsigned nb = nblk(N, kWG);
    const unsigned gstride = nb < 4096u ? nb : 4096u;
    const int selfscan = (nb <= (unsigned)kSelfScanMax) ? 1 : 0;
    if (!selfscan)
        TDE_LAUNCH(k_scan_blocks, 1, 1024, stream, (const int*)wl.bsumA, wl.bsum, (const int*)nullptr, (int*)nullptr,
                   (int)nb);
    TDE_LAUNCH(k_nncompact, nb, kWG, stream, N, wl, selfscan);
    TDE_LAUNCH(k_runs, gstride, kWG, stream, mr, blkm, N, wl);
    if (!selfscan)
        TDE_LAUNCH(k_scan_blocks, 1, 1024, stream, (const int*)wl.bsumA, wl.bsumAs, (const int*)wl.bsumR, wl.bsumRs,
                   (int)nb);
    TDE_LAUNCH(k_actcompact, nb, kWG, stream, mr, blkm, N, wl, selfscan);
}

// This level's slice of the per-level block counters.
static Work level_work(const Work& w, long long ntot, size_t h) {
    const long long nbs = (ntot + kWG - 1) / kWG + 2;
    Work wl = w;
    wl.bsumA = w.bcnt + (long long)h * 2 * nbs;
    wl.bsumR = wl.bsumA + nbs;
    return wl;
}

static long long bcnt_entries(const Plan& p) { return (long long)p.levels.size() * 2 * ((p.ntot + kWG - 1) / kWG + 2); }

static void enqueue_setup(const Plan& p, const Work& w, void* stream) {
    const long long nbc = p.levels.empty() ? 0 : bcnt_entries(p);
    const long long ncnt = (long long)CNT_N * kCntSlots;
    long long most = nbc > p.B ? nbc : p.B;
    if (most < ncnt) most = ncnt;
    unsigned g = nblk(most, kWG);
    if (g > 64) g = 64;
    TDE_LAUNCH_K(KIND_SETUP, k_setup, g, kWG, stream, w.status, 16LL, w.counters, ncnt, w.pmax, (long long)p.B,
                 w.bcnt, nbc);
}

// QL leaves per wave: 64, or for fewer than 64 * kLeafWaves leaves the
// largest power of two that still gives kLeafWaves waves (at least one leaf).
// Spreading a handful of leaves over more waves shortens the solve (n = 1024
// in leaves of 32: 1.0 -> 0.68 ms for the leaves); spreading thousands over
// one wave per SIMD lengthens it (4096 leaves of 16: 0.30 -> 0.43 ms).
constexpr int kLeafWaves = 64;
static int leaves_per_wave(int nleaves) {
    int per = 64;
    while (per > 1 && (long long)nleaves < (long long)per * kLeafWaves) per >>= 1;
    return per;
}

int enqueue_solve(const Plan& p, const Work& w, const double* d, const double* e, double* out, void* stream,
                  const Ckpt* ck, const Ckpt* xsrc) {
    if (p.ntot == 0) return 0;
    enqueue_setup(p, w, stream);
    TDE_LAUNCH_K(KIND_SETUP, k_maxabs, nblk(p.ntot, kWG * kMaxAbsPer), kWG, stream, d, e, (const long long*)p.d_offs, p.B,
                 p.ntot, w.pmax, w.status);
    if (p.nleaves > 0 && p.leaf_dc && !ck) {
        // the checkpointing forward keeps the QL leaves the reverse pass differentiates
        TDE_LAUNCH_K(KIND_LEAF, k_leaf_dc, (unsigned)p.nleaves, 64, stream, p.d_leaves, p.d_shdr, p.d_smer, d, e,
                     (const unsigned long long*)w.pmax, w, out);
    } else if (p.nleaves > 0) {
        const int per = leaves_per_wave(p.nleaves);
        const unsigned g = nblk(p.nleaves, per);
        if (p.leafmax <= 8)
            TDE_LAUNCH_K(KIND_LEAF, k_leaf<8>, g, 64, stream, p.d_leaves, p.nleaves, d, e, w.pmax, w, out, per);
        else if (p.leafmax <= 16)
            TDE_LAUNCH_K(KIND_LEAF, k_leaf<16>, g, 64, stream, p.d_leaves, p.nleaves, d, e, w.pmax, w, out, per);
        else if (p.leafmax <= 32)
            TDE_LAUNCH_K(KIND_LEAF, k_leaf<32>, g, 64, stream, p.d_leaves, p.nleaves, d, e, w.pmax, w, out, per);
        else
            TDE_LAUNCH_K(KIND_LEAF, k_leaf<64>, g, 64, stream, p.d_leaves, p.nleaves, d, e, w.pmax, w, out, per);
    }
    for (size_t h = 0; h < p.levels.size(); ++h) {
        const LevelInfo& L = p.levels[h];
        const MergeRec* mr = p.d_merges + L.mstart;
        const int* blkm = p.d_blkm + L.bstart;
        const int M = L.M;
        const long long N = L.N;
        const unsigned nb = nblk(N, kWG);
        Work wl = level_work(w, p.ntot, h);
        if (xsrc) {
            // requested-rows pass: the level's node spectra and boundary rows from the checkpoint
            const long long so = (long long)h * xsrc->n;
            wl.lam = xsrc->lam + so;
            wl.blo = xsrc->blo + so;
            wl.bhi = xsrc->bhi + so;
        }
        if (ck) {
            const long long so = (long long)h * ck->n;
            TDE_LAUNCH_K(KIND_SETUP, k_ckpt_save, nb, kWG, stream, mr, blkm, N, w, ck->lam + so, ck->blo + so,
                         ck->bhi + so);
            wl.org = ck->org + so;
            wl.tau = ck->tau + so;
        }
        if (level_blocked(L)) {
            // every merge of the level fits one workgroup (or a pack of them one
            // wave): the whole merge in one launch (with a checkpoint, its roots
            // land at the merge's packed positions)
            if (level_waved(L) && !w.rows_out && !xsrc && L.smax <= 32)
                TDE_LAUNCH_K(KIND_LEVEL, k_level_wave<1>, (unsigned)L.nwp, 64, stream, mr, p.d_blkm + L.wpstart, e,
                             (const unsigned long long*)w.pmax, wl, out, ck ? 1 : 0);
            else if (level_waved(L) && !w.rows_out && !xsrc)
                TDE_LAUNCH_K(KIND_LEVEL, k_level_wave<4>, (unsigned)L.nwp, 64, stream, mr, p.d_blkm + L.wpstart, e,
                             (const unsigned long long*)w.pmax, wl, out, ck ? 1 : 0);
            else
                launch_level_block(L.smax, mr, M, e, wl, out, fused_gmax(M, p.group_max), stream);
            continue;
        }
        launch_merge(KIND_MERGE, L, mr, blkm, e, wl, stream);
        enqueue_deflate(mr, blkm, N, wl, stream);
        const bool placed = launch_roots(L.smax, p.sweep_cols, p.wide_min, N, mr, blkm, M, e, wl, out,
                                         fused_gmax(M, p.group_max),
                                         p.wide_blocks > 0 ? p.wide_blocks : (int)kWideGridMax, p.fuse_few,
                                         L.all_root && !w.rows_out, stream);
        if (placed)
            continue;
        else if (N <= kWideSearchCols)
            TDE_LAUNCH_K(KIND_ASSEMBLE, k_assemble<true>, nb, kWG, stream, mr, blkm, N,
                         (const unsigned long long*)w.pmax, wl, out);
        else
            TDE_LAUNCH_K(KIND_ASSEMBLE, k_assemble<false>, nb, kWG, stream, mr, blkm, N,
                         (const unsigned long long*)w.pmax, wl, out);
    }
    return (int)hipGetLastError();
}

// Reverse pass of a level's roots: z-hat recomputed from the checkpointed
// roots together with the unassembly of the parent's adjoints (one launch),
// then the per-root coefficients and the per-pole adjoints.
template <int G>
static void launch_bwd_roots_g(int smax, int wmin, long long N, const MergeRec* mr, const int* blkm, int M,
                               const double* e, const Work& w, const Grad& gr, long long cs, void* stream) {
    const bool wide = smax >= wmin;
    const int wide_min = wide ? wmin : 0x7fffffff;
    int nbn, nbw;
    root_grid(N, G, wide, &nbn, &nbw);
    const unsigned long long* pm = (const unsigned long long*)w.pmax;
    const unsigned nbu = nblk(N, kWG);
    if (wide) TDE_LAUNCH_K(KIND_BACKWARD, k_wide_items, 1, 1024, stream, mr, M, w, wide_min, 0);
    TDE_LAUNCH_K(KIND_BACKWARD, (k_lowner<G, true>), (unsigned)(nbn + nbw) + nbu, kWG, stream, mr, M, N, e, pm, w,
                 wide_min, 0, nbn, blkm, gr, (int)nbu, N <= kWideSearchCols ? 1 : 0, (double*)nullptr);
    TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_roots<G>, (unsigned)nbn, kWG, stream, mr, N, w, gr, cs);
    TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_poles<G>, (unsigned)nbn, kWG, stream, mr, N, w, gr, cs);
}

// The couplings deflation drops (negligible columns, rotated runs, G lanes
// per column or run) and the merges' dL/drho~, one launch.
template <int G>
static void launch_bwd_defl(long long N, int M, const MergeRec* mr, const int* blkm, const double* e,
                            const Work& w, const Grad& gr, long long cs, int mstart, void* stream) {
    const unsigned nbr = nblk(N, kWG) < 4096u ? nblk(N, kWG) : 4096u;
    const unsigned nbn = nblk(N * G, kWG);
    TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_defl<G>, nbr + nbn + (unsigned)M, kWG, stream, mr, blkm, N, e,
                 (const unsigned long long*)w.pmax, w, gr, cs, mstart, (int)nbr, (int)nbn);
}

int enqueue_backward(const Plan& p, const Work& w, const Grad& gr, const Ckpt& ck, const double* d,
                     const double* e, const double* gin, double* gd, double* ge, void* stream) {
    if (p.ntot == 0) return 0;
    const long long cs = p.ntot;  // coefficient plane stride
    enqueue_setup(p, w, stream);
    TDE_LAUNCH_K(KIND_SETUP, k_maxabs, nblk(p.ntot, kWG * kMaxAbsPer), kWG, stream, d, e, (const long long*)p.d_offs, p.B,
                 p.ntot, w.pmax, w.status);
    TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_init, nblk(p.ntot, kWG), kWG, stream, p.ntot, gin, gr);
    for (size_t hh = p.levels.size(); hh-- > 0;) {
        const LevelInfo& L = p.levels[hh];
        const MergeRec* mr = p.d_merges + L.mstart;
        const int* blkm = p.d_blkm + L.bstart;
        const int M = L.M;
        const long long N = L.N;
        const unsigned nb = nblk(N, kWG);
        const long long so = (long long)hh * ck.n;
        Work wl = level_work(w, p.ntot, hh);
        wl.lam = ck.lam + so;
        wl.blo = ck.blo + so;
        wl.bhi = ck.bhi + so;
        wl.org = ck.org + so;
        wl.tau = ck.tau + so;
        launch_merge(KIND_BACKWARD, L, mr, blkm, e, wl, stream);
        enqueue_deflate(mr, blkm, N, wl, stream);
        if (level_blocked(L)) {
            wl.org = w.org;
            wl.tau = w.tau;
            TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_roots_gather, nb < 4096u ? nb : 4096u, kWG, stream, mr, N, wl,
                         (const int*)(ck.org + so), (const double*)(ck.tau + so));
        }
        switch (lanes_per_root(L.smax, p.sweep_cols)) {
            case 1: launch_bwd_roots_g<1>(L.smax, p.wide_min, N, mr, blkm, M, e, wl, gr, cs, stream); break;
            case 2: launch_bwd_roots_g<2>(L.smax, p.wide_min, N, mr, blkm, M, e, wl, gr, cs, stream); break;
            case 4: launch_bwd_roots_g<4>(L.smax, p.wide_min, N, mr, blkm, M, e, wl, gr, cs, stream); break;
            case 8: launch_bwd_roots_g<8>(L.smax, p.wide_min, N, mr, blkm, M, e, wl, gr, cs, stream); break;
            default: launch_bwd_roots_g<16>(L.smax, p.wide_min, N, mr, blkm, M, e, wl, gr, cs, stream); break;
        }
        switch (lanes_per_root(L.smax, p.sweep_cols)) {
            case 1: launch_bwd_defl<1>(N, M, mr, blkm, e, wl, gr, cs, L.mstart, stream); break;
            case 2: launch_bwd_defl<2>(N, M, mr, blkm, e, wl, gr, cs, L.mstart, stream); break;
            case 4: launch_bwd_defl<4>(N, M, mr, blkm, e, wl, gr, cs, L.mstart, stream); break;
            case 8: launch_bwd_defl<8>(N, M, mr, blkm, e, wl, gr, cs, L.mstart, stream); break;
            default: launch_bwd_defl<16>(N, M, mr, blkm, e, wl, gr, cs, L.mstart, stream); break;
        }
        TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_merge, nb, kWG, stream, mr, blkm, N, e, (const unsigned long long*)w.pmax,
                     wl, gr);
    }
    if (p.nleaves > 0) {
        if (p.leafmax <= 8)
            TDE_LAUNCH_K(KIND_BACKWARD, (k_bwd_leaf<8, 2>), nblk(p.nleaves, 16), 64, stream, p.d_leaves, p.nleaves, d,
                         e, w.pmax, w, gr, gd, ge);
        else if (p.leafmax <= 16)
            TDE_LAUNCH_K(KIND_BACKWARD, (k_bwd_leaf<16, 1>), nblk(p.nleaves, 4), 64, stream, p.d_leaves, p.nleaves, d,
                         e, w.pmax, w, gr, gd, ge);
        else if (p.leafmax <= 32)
            TDE_LAUNCH_K(KIND_BACKWARD, (k_bwd_leaf<32, 1>), nblk(p.nleaves, 2), 64, stream, p.d_leaves, p.nleaves, d,
                         e, w.pmax, w, gr, gd, ge);
        else
            TDE_LAUNCH_K(KIND_BACKWARD, (k_bwd_leaf<64, 1>), (unsigned)p.nleaves, 64, stream, p.d_leaves, p.nleaves,
                         d, e, w.pmax, w, gr, gd, ge);
    }
    if (p.nmerges > 0)
        TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_tear, nblk(p.nmerges, kWG), kWG, stream, p.d_merges, p.nmerges, e,
                     (const unsigned long long*)w.pmax, gr, ge);
    TDE_LAUNCH_K(KIND_BACKWARD, k_bwd_edges, nblk(p.B, kWG), kWG, stream, (const long long*)p.d_offs, p.B, ge);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Driver pre-pass: split at negligible couplings (the outer structure of a
// tridiagonal eigensolver driver: independent unreduced blocks, each scaled
// on its own), and the merge of the blocks' ascending spectra afterwards.
// ---------------------------------------------------------------------------

// flags[i] = 1 when the coupling e[i-1] is negligible beside its diagonal
// neighbours, |e| <= eps sqrt|d_{i-1}| sqrt|d_i| (setting it to zero moves no
// eigenvalue by more than eps ||T||), for 1 <= i < n; flags[0] = 1.  Problem
// starts are added by the host, so the unused slot e[off_b - 1] of the
// batched layout is read but never decides anything.
__global__ __launch_bounds__(kWG) void k_split_flags(const double* __restrict__ d, const double* __restrict__ e,
                                                     long long n, int* __restrict__ flags) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) {
        flags[0] = 1;
        return;
    }
    const double tiny = DBL_EPSILON * sqrt(fabs(d[i - 1])) * sqrt(fabs(d[i]));
    flags[i] = (fabs(e[i - 1]) <= tiny) ? 1 : 0;
}

// One pass of the pairwise merges of ascending runs: merge m combines the
// adjacent runs [off, off + nL) and [off + nL, off + nL + nR) of src into the
// same range of dst (ties: left run first); columns in no merge of this pass
// are copied.  recs are sorted by off.
__global__ __launch_bounds__(kWG) void k_merge_runs(const MergeRec* __restrict__ recs, int M,
                                                    const double* __restrict__ src, double* __restrict__ dst,
                                                    long long n) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (recs[mid].off <= t) lo = mid;
        else hi = mid - 1;
    }
    const MergeRec R = recs[lo];
    const double x = src[t];
    if (t < R.off || t >= R.off + R.nL + R.nR) {
        dst[t] = x;
        return;
    }
    const int i = (int)(t - R.off);
    int pos;
    if (i < R.nL) pos = i + count_lt(src + R.off + R.nL, R.nR, x);
    else pos = (i - R.nL) + count_le(src + R.off, R.nL, x);
    dst[R.off + pos] = x;
}

int enqueue_selrows_fix(double* Q, long long m, long long n, const int* first, const double* q0,
                        const double* q1, void* stream) {
    if (m <= 0 || n <= 0) return 0;
    TDE_LAUNCH_K(KIND_ASSEMBLE, k_selrows_fix, nblk(n, kWG), kWG, stream, Q, m, n, first, q0, q1);
    return (int)hipGetLastError();
}

int enqueue_split_flags(const double* d, const double* e, long long n, int* flags, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_split_flags, dim3(nblk(n, kWG)), dim3(kWG), 0, (hipStream_t)stream, d, e, n, flags);
    return (int)hipGetLastError();
}

int enqueue_merge_runs(const MergeRec* recs, int M, const double* src, double* dst, long long n, void* stream) {
    if (n <= 0 || M <= 0) return 0;
    hipLaunchKernelGGL(k_merge_runs, dim3(nblk(n, kWG)), dim3(kWG), 0, (hipStream_t)stream, recs, M, src, dst, n);
    return (int)hipGetLastError();
}

}  // namespace tde
