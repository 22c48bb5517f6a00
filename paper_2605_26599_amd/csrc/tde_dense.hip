// Dense front end: reduction of a real symmetric matrix to tridiagonal form
// on the MI355X, then the boundary-row solve of the tridiagonal.
//
// Dense symmetric EVD first reduces A to T = Q^T A Q by orthogonal
// transformations (the eigenvalues of T are those of A) and then solves the
// tridiagonal problem (Section 2.1); for eigenvalues only the transformations
// are not kept.  The reduction here is the blocked Householder scheme of
// LAPACK's symmetric tridiagonal reduction (lower triangle, panel width kNb):
// inside a panel, column c is brought up to date with the panel's earlier
// reflectors, its reflector v (v_0 = 1) and tau are formed, and
// w = tau (A22 v - V (W^T v) - W (V^T v)) + alpha v with
// alpha = -tau/2 (w^T v) is taken against the trailing matrix as it stood at
// the start of the panel; after the panel the trailing matrix receives the
// rank-2b update A22 <- A22 - V W^T - W V^T as one matrix product on the FP64
// matrix cores.  A is kept in full (both triangles), so the per-column
// product A22 v reads whole columns (contiguous in memory, column-major):
// y_r = A[:, r] . v, one wave per column r.
//
// Per column three launches, each spread over the whole chip: k_trd_symv
// (one wave per trailing column, plus one per dot product W^T v, V^T v),
// k_trd_wrow (w row by row) and k_trd_colx (the next column brought up to
// date and its reflector formed, row by row); per panel k_trd_colx for its
// first column, k_trd_wfix after its last column, and k_trd_syr2k.  The two
// row-parallel kernels end in a reduction (w^T v, the column's norm): every
// workgroup stores its partial sum, and the last one to finish (an atomic
// ticket, no waiting) adds the partials in workgroup order and forms the
// scalars, so the result does not depend on which workgroup finishes last;
// the next launch applies them to the column (the reflector's scale in
// k_trd_symv, w's alpha v in the next k_trd_colx).
// The memory traffic is dominated by the trailing-matrix reads of k_trd_symv
// (about 8 n^3 / 3 bytes in all); the panel products are about 4 n^3 / 3
// FLOP on the matrix cores (both triangles).
#include <hip/hip_runtime.h>

#include "tde_dense.h"

namespace tde {

namespace {

constexpr int kRowThreads = 128;  // rows per workgroup of the row-parallel kernels

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup (every thread gets it); red: one double per wave.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += red[k];  // fixed order: every thread the same bits
    return t;
}

// The workgroup's partial sum goes to part[blockIdx.x]; returns true in the
// last workgroup to arrive (every thread of it), which then sees every
// partial.  The ticket is left at zero for the next use.
__device__ __forceinline__ bool arrive_last(double partial, double* __restrict__ part,
                                            unsigned* __restrict__ ticket, bool* s_last) {
    if (threadIdx.x == 0) {
        part[blockIdx.x] = partial;
        __threadfence();
        const unsigned k = atomicAdd(ticket, 1u);
        *s_last = (k == gridDim.x - 1);
        if (*s_last) *ticket = 0u;
    }
    __syncthreads();
    const bool last = *s_last;
    if (last) __threadfence();
    return last;
}

// Sum of part[0..nb) in workgroup order (the same bits whoever is last),
// every thread of the workgroup; the partials pass through LDS so that their
// loads are in flight together.
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int nb, double* sp) {
    double t = 0.0;
    for (int b0 = 0; b0 < nb; b0 += kRowThreads) {
        if (b0 + (int)threadIdx.x < nb) sp[threadIdx.x] = part[b0 + threadIdx.x];
        __syncthreads();
        const int cnt = (nb - b0 < kRowThreads) ? nb - b0 : kRowThreads;
        for (int k = 0; k < cnt; ++k) t += sp[k];
        __syncthreads();
    }
    return t;
}

// Column c, with the panel's first i reflectors: rows c..n-1 brought up to
// date (a = A[:, c] - V W[c, :]^T - W V[c, :]^T), the diagonal entry
// recorded, and the reflector of rows c+1..n-1 formed: its entries unscaled
// in ua (ua[c+1] = alpha), tau[i], e[c] = beta and the scale of the other
// entries in sc[0] (v = ua sc[0], v_(c+1) = 1; k_trd_symv stores v as column
// i of V).  With i > 0 the previous column's w is completed on the way: its
// rows below c receive alpha v (alpha = sc[1], from k_trd_wrow), row c is
// used completed and never read again.  One thread per row; the last
// workgroup forms the reflector from the norm.
__global__ __launch_bounds__(kRowThreads) void k_trd_colx(const double* __restrict__ A, long long lda, int n, int c,
                                                         int i, const double* __restrict__ V,
                                                         double* __restrict__ W, double* __restrict__ ua,
                                                         double* __restrict__ tau, double* __restrict__ d,
                                                         double* __restrict__ e, double* __restrict__ sc,
                                                         double* __restrict__ part, unsigned* __restrict__ ticket) {
    __shared__ double red[kRowThreads / 64];
    __shared__ bool s_last;
    const long long ln = n;
    const int r = c + (int)(blockIdx.x * kRowThreads + threadIdx.x);
    const int jl = i - 1;  // the previous column (i > 0)
    const double alpha = (i > 0) ? sc[1] : 0.0;
    const double wlc = (i > 0) ? fma(alpha, V[jl * ln + c], W[jl * ln + c]) : 0.0;
    double ssq = 0.0;
    if (r < n) {
        double a = A[(long long)c * lda + r];
        // unrolled so that eight reflectors' loads are in flight together
#pragma unroll 8
        for (int j = 0; j < jl; ++j) a -= V[j * ln + r] * W[j * ln + c] + W[j * ln + r] * V[j * ln + c];
        if (i > 0) {
            const double wr = (r == c) ? wlc : fma(alpha, V[jl * ln + r], W[jl * ln + r]);
            if (r > c) W[jl * ln + r] = wr;
            a -= V[jl * ln + r] * wlc + wr * V[jl * ln + c];
        }
        if (r == c) d[c] = a;
        else ua[r] = a;
        if (r >= c + 2) ssq = a * a;
    }
    const double bs = block_sum<kRowThreads>(ssq, red);
    if (!arrive_last(bs, part, ticket, &s_last)) return;  // workgroup-uniform
    __shared__ double sp[kRowThreads];
    const double xn2 = sum_parts(part, (int)gridDim.x, sp);
    if (threadIdx.x == 0) {
        const double ah = ua[c + 1];
        double t = 0.0, scale = 0.0, beta = ah;
        if (xn2 > 0.0) {
            const double nrm = sqrt(fma(ah, ah, xn2));
            beta = (ah >= 0.0) ? -nrm : nrm;
            t = (beta - ah) / beta;
            scale = 1.0 / (ah - beta);
        }
        tau[i] = t;
        e[c] = beta;
        sc[0] = scale;
    }
}

// y_r = A[c+1:, r] . v for every trailing column r (symmetric A: column r
// holds row r), one wave per column; then one wave per dot product
// sdot[q] = W_q . v (q < i) and sdot[i + q] = V_q . v over the same rows.
// v = ua sc[0] with v_(c+1) = 1 (k_trd_colx's reflector); the wave of
// column r also stores v_r into column i of V.
__global__ __launch_bounds__(256) void k_trd_symv(const double* __restrict__ A, long long lda, int n, int c, int i,
                                                 double* __restrict__ V, const double* __restrict__ W,
                                                 const double* __restrict__ ua, const double* __restrict__ sc,
                                                 double* __restrict__ y, double* __restrict__ sdot) {
    const int j = (int)((blockIdx.x * 256 + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    const int m = n - c - 1;
    if (j >= m + 2 * i) return;  // wave-uniform
    const double scale = sc[0];
    const double* __restrict__ u;
    if (j < m) u = A + (long long)(c + 1 + j) * lda;
    else u = (j - m < i) ? W + (long long)(j - m) * n : V + (long long)(j - m - i) * n;
    auto vk = [&](int k) { return (k == c + 1) ? 1.0 : ua[k] * scale; };
    double acc0 = 0.0, acc1 = 0.0;
    int k = c + 1 + lane;
    for (; k + 64 < n; k += 128) {
        acc0 = fma(u[k], vk(k), acc0);
        acc1 = fma(u[k + 64], vk(k + 64), acc1);
    }
    if (k < n) acc0 = fma(u[k], vk(k), acc0);
    const double s = wave_sum(acc0 + acc1);
    if (lane == 0) {
        if (j < m) {
            y[c + 1 + j] = s;
            V[(long long)i * n + c + 1 + j] = vk(c + 1 + j);
        } else {
            sdot[j - m] = s;
        }
    }
}

// w' = tau (y - V (W^T v) - W (V^T v)) over rows c+1..n-1, one thread per
// row, stored as column i of W; the last workgroup forms alpha = -tau/2
// (w'^T v) into sc[1].  w = w' + alpha v is completed by the next column's
// k_trd_colx, or by k_trd_wfix after a panel's last column.
__global__ __launch_bounds__(kRowThreads) void k_trd_wrow(int n, int c, int i, const double* __restrict__ V,
                                                         double* __restrict__ W, const double* __restrict__ y,
                                                         const double* __restrict__ tau,
                                                         const double* __restrict__ sdot, double* __restrict__ sc,
                                                         double* __restrict__ part, unsigned* __restrict__ ticket) {
    __shared__ double red[kRowThreads / 64];
    __shared__ bool s_last;
    const long long ln = n;
    const double t = tau[i];
    const int r = c + 1 + (int)(blockIdx.x * kRowThreads + threadIdx.x);
    double wv = 0.0;
    if (r < n) {
        double a = y[r];
#pragma unroll 8
        for (int j = 0; j < i; ++j) a -= V[j * ln + r] * sdot[j] + W[j * ln + r] * sdot[i + j];
        a *= t;
        W[i * ln + r] = a;
        wv = a * V[i * ln + r];
    }
    const double bs = block_sum<kRowThreads>(wv, red);
    if (!arrive_last(bs, part, ticket, &s_last)) return;  // workgroup-uniform
    __shared__ double sp[kRowThreads];
    const double alpha = -0.5 * t * sum_parts(part, (int)gridDim.x, sp);
    if (threadIdx.x == 0) sc[1] = alpha;
}

// w = w' + alpha v for column i of W, rows c+1..n-1 (after a panel's last column).
__global__ __launch_bounds__(kRowThreads) void k_trd_wfix(int n, int c, int i, const double* __restrict__ V,
                                                         double* __restrict__ W, const double* __restrict__ sc) {
    const long long ln = n;
    const int r = c + 1 + (int)(blockIdx.x * kRowThreads + threadIdx.x);
    if (r < n) W[i * ln + r] = fma(sc[1], V[i * ln + r], W[i * ln + r]);
}

__global__ void k_trd_zero(unsigned* __restrict__ ticket) {
    if (threadIdx.x < 2) ticket[threadIdx.x] = 0u;
}

// Trailing update A[q:, q:] -= V W^T + W V^T (rows and columns q..n-1, both
// triangles) on the FP64 matrix cores.  With U = [V | W] and Z = [W | V]
// (n x 2b) the update is U Z^T.  One wave per 32 x 32 tile of A, as 2 x 2
// blocks of V_MFMA_F64_16X16X4F64 (D = A_op B_op + C, A_op 16 x 4, B_op
// 4 x 16): A_op[i][k] = Z[s0 + i][k], B_op[k][j] = U[r0 + j][k], so
// D[i][j] is the update of A[r0 + j][s0 + i]; lane l supplies A_op[l % 16][l / 16]
// and B_op[l / 16][l % 16] and holds D[4 t + l / 16][l % 16] in its register
// t = 0..3, i.e. row r0 + l % 16 of column s0 + 4 t + l / 16: sixteen lanes
// touch sixteen consecutive rows of one column.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_trd_syr2k(double* __restrict__ A, long long lda, int n, int q, int b,
                                                  const double* __restrict__ V, const double* __restrict__ W,
                                                  int tiles) {
    const int wave = (int)((blockIdx.x * 256 + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    const int tr = wave % tiles, tc = wave / tiles;
    if (tc >= tiles) return;  // wave-uniform
    const int r0 = q + 32 * tr, s0 = q + 32 * tc;
    const long long ln = n;
    const int li = lane & 15, lk = lane >> 4;
    v4d acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) acc[a][bb] = v4d{0.0, 0.0, 0.0, 0.0};
    // rows of this lane's operands (out-of-range rows contribute zero)
    const int sr0 = s0 + li, sr1 = s0 + 16 + li;  // Z rows (A operand), blocks ib = 0, 1
    const int ur0 = r0 + li, ur1 = r0 + 16 + li;  // U rows (B operand), blocks jb = 0, 1
    for (int k0 = 0; k0 < 2 * b; k0 += 4) {
        const int k = k0 + lk;
        double za0 = 0.0, za1 = 0.0, ub0 = 0.0, ub1 = 0.0;
        if (k < 2 * b) {
            // Z = [W | V], U = [V | W]
            const double* __restrict__ zc = (k < b) ? W + (long long)k * ln : V + (long long)(k - b) * ln;
            const double* __restrict__ uc = (k < b) ? V + (long long)k * ln : W + (long long)(k - b) * ln;
            if (sr0 < n) za0 = zc[sr0];
            if (sr1 < n) za1 = zc[sr1];
            if (ur0 < n) ub0 = uc[ur0];
            if (ur1 < n) ub1 = uc[ur1];
        }
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(za0, ub0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(za0, ub1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(za1, ub0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(za1, ub1, acc[1][1], 0, 0, 0);
    }
    for (int ib = 0; ib < 2; ++ib)
        for (int jb = 0; jb < 2; ++jb) {
            const int r = r0 + 16 * jb + li;
            if (r >= n) continue;
            for (int t = 0; t < 4; ++t) {
                const int s = s0 + 16 * ib + 4 * t + lk;
                if (s < n) A[(long long)s * lda + r] -= acc[ib][jb][t];
            }
        }
}

// The last 2 x 2 (or 1 x 1) block after every update.
__global__ void k_trd_tail(const double* __restrict__ A, long long lda, int n, double* __restrict__ d,
                           double* __restrict__ e) {
    if (threadIdx.x != 0 || n < 1) return;
    if (n == 1) {
        d[0] = A[0];
        return;
    }
    d[n - 2] = A[(long long)(n - 2) * lda + (n - 2)];
    d[n - 1] = A[(long long)(n - 1) * lda + (n - 1)];
    e[n - 2] = A[(long long)(n - 2) * lda + (n - 1)];
}

}  // namespace

size_t dense_layout(long long n, char* base, DenseWork* dw) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const long long nn = n > 0 ? n : 1;
    DenseWork t{};
    t.V = (double*)take(8 * nn * kNb);
    t.W = (double*)take(8 * nn * kNb);
    t.y = (double*)take(8 * nn);
    t.tau = (double*)take(8 * kNb);
    t.sdot = (double*)take(8 * 2 * kNb);
    t.ua = (double*)take(8 * nn);
    t.sc = (double*)take(8 * 2);
    t.part = (double*)take(8 * (nn / kRowThreads + 2));
    t.ticket = (unsigned*)take(8);
    t.d = (double*)take(8 * nn);
    t.e = (double*)take(8 * nn);
    if (dw) *dw = t;
    return off;
}

int enqueue_dense_reduce(double* A, long long lda, int n, const DenseWork& dw, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_trd_zero, dim3(1), dim3(64), 0, s, dw.ticket);
    auto rows = [](int count) { return dim3((unsigned)((count + kRowThreads - 1) / kRowThreads)); };
    for (int p = 0; p < n - 2; p += kNb) {
        const int b = (n - 2 - p < kNb) ? n - 2 - p : kNb;
        hipLaunchKernelGGL(k_trd_colx, rows(n - p), dim3(kRowThreads), 0, s, A, lda, n, p, 0, dw.V, dw.W, dw.ua,
                           dw.tau, dw.d, dw.e, dw.sc, dw.part, dw.ticket);
        for (int i = 0; i < b; ++i) {
            const int c = p + i;
            const int m = n - c - 1;  // trailing columns
            hipLaunchKernelGGL(k_trd_symv, dim3((unsigned)((m + 2 * i + 3) / 4)), dim3(256), 0, s, A, lda, n, c, i,
                               dw.V, dw.W, dw.ua, dw.sc, dw.y, dw.sdot);
            hipLaunchKernelGGL(k_trd_wrow, rows(m), dim3(kRowThreads), 0, s, n, c, i, dw.V, dw.W, dw.y, dw.tau,
                               dw.sdot, dw.sc, dw.part, dw.ticket);
            if (i + 1 < b)
                hipLaunchKernelGGL(k_trd_colx, rows(n - c - 1), dim3(kRowThreads), 0, s, A, lda, n, c + 1, i + 1,
                                   dw.V, dw.W, dw.ua, dw.tau, dw.d, dw.e, dw.sc, dw.part, dw.ticket + 1);
            else
                hipLaunchKernelGGL(k_trd_wfix, rows(m), dim3(kRowThreads), 0, s, n, c, i, dw.V, dw.W, dw.sc);
        }
        const int q = p + b;
        const int M = n - q;
        const int tiles = (M + 31) / 32;
        const long long waves = (long long)tiles * tiles;
        hipLaunchKernelGGL(k_trd_syr2k, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, A, lda, n, q, b, dw.V,
                           dw.W, tiles);
    }
    hipLaunchKernelGGL(k_trd_tail, dim3(1), dim3(64), 0, s, A, lda, n, dw.d, dw.e);
    return (int)hipGetLastError();
}

}  // namespace tde
