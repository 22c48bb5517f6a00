// Boundary-row divide and conquer on the host CPU: the paper's CPU design
// (Section 4.2) as a second host baseline beside the GPU library.  It is a
// separate program: it shares no code with the HIP kernels or the oracle and
// is never called by the GPU entry points.
//
// Driver (Section 4.2): validate, split at negligible couplings, scale every
// unreduced block by a power of two, solve small blocks by implicit QR and
// larger ones by BR D&C, and sort the union of the blocks' spectra.
// BR D&C (Algorithm 1): a balanced split tree down to leaves of at most 32
// columns; every leaf solved by implicit QR tracking only its first and last
// eigenvector rows (Lemma 2); merges level by level, the merges of one level
// in parallel (OpenMP) with disjoint workspace slices given by their column
// ranges; a level with fewer merges than threads parallelises inside each
// merge (roots, Loewner products, rows).  Per merge (Section 3.1, Eq.
// merge-problem): z = [last row of Q_L; sign(beta) first row of Q_R]/sqrt 2
// with rho = 2|beta|, merge of the two ascending child spectra, deflation of
// negligible z and close poles (Givens rotations applied to D, z and both
// outer rows), secular roots in compact (origin pole, offset) form (Section
// 4.1; appendix on compact denominators), Loewner-recomputed z and the
// parent's first and last rows as two streamed dot products per root
// (Section 3.2, Eq. boundary-state); the top merge skips the rows (root-only
// mode, Section 3.3).  Workspace: 16 n doubles and 2 n ints, carved by column
// range (no K x K block, nothing per thread).
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "../../include/tde_host.h"

namespace {

constexpr int kLeaf = 32;      // largest leaf of the split tree
constexpr int kQrCap = 40;     // implicit QR steps allowed per eigenvalue
constexpr int kSecCap = 100;   // secular iterations allowed per root

// ---------------------------------------------------------------------------
// Implicit symmetric QR with a Wilkinson shift (Golub and Van Loan, Matrix
// Computations, Algorithm 8.3.2: shift from the trailing 2x2 block, bulge
// chased downward), optionally tracking the first and last rows of the
// eigenvector matrix Z (Z <- Z P^T for every plane rotation P).
//
// Plane rotation P = [c s; -s c] in rows/columns (k, k+1) of T, applied as
// P T P^T: with the block [p r; r q], w = s (q - p) + 2 c r gives
// p' = p + s w, q' = q - s w, r' = c w - r (c^2 + s^2 = 1; trace kept); the
// entry below, b_(k+1), becomes c b_(k+1) and leaves the bulge s b_(k+1) at
// (k+2, k).  Rows of Z: (z_k, z_(k+1)) <- (c z_k + s z_(k+1), c z_(k+1) - s z_k).
// ---------------------------------------------------------------------------
struct QrRows {
    double* r0;  // first row of Z, or null
    double* r1;  // last row of Z, or null
};

int qr_solve(int n, double* a, double* b, QrRows rows) {
    // a[0..n) diagonal, b[0..n-1) couplings (destroyed); a returns the
    // eigenvalues ascending, the tracked rows permuted alongside
    if (rows.r0)
        for (int i = 0; i < n; ++i) rows.r0[i] = (i == 0) ? 1.0 : 0.0;
    if (rows.r1)
        for (int i = 0; i < n; ++i) rows.r1[i] = (i == n - 1) ? 1.0 : 0.0;
    auto negligible = [&](int k) { return fabs(b[k]) <= DBL_EPSILON * (fabs(a[k]) + fabs(a[k + 1])); };
    int status = 0;
    int m = n - 1, steps = 0;
    while (m > 0) {
        if (negligible(m - 1)) {
            b[m - 1] = 0.0;
            --m;
            steps = 0;
            continue;
        }
        int l = m - 1;
        while (l > 0 && !negligible(l - 1)) --l;
        if (l > 0) b[l - 1] = 0.0;
        if (++steps > kQrCap) {
            status = 1;
            b[m - 1] = 0.0;  // give up on this eigenvalue
            --m;
            steps = 0;
            continue;
        }
        // Wilkinson shift: eigenvalue of the trailing 2x2 block nearer to a[m]
        const double t = 0.5 * (a[m - 1] - a[m]);
        const double bm = b[m - 1];
        const double den = t + (t >= 0.0 ? hypot(t, bm) : -hypot(t, bm));
        const double mu = (den == 0.0) ? a[m] - fabs(bm) : a[m] - bm * (bm / den);
        double x = a[l] - mu, z = b[l];
        for (int k = l; k < m; ++k) {
            const double h = hypot(x, z);
            const double c = (h == 0.0) ? 1.0 : x / h;
            const double s = (h == 0.0) ? 0.0 : z / h;
            if (k > l) b[k - 1] = h;  // the bulge is gone
            const double p = a[k], q = a[k + 1], r = b[k];
            const double w = s * (q - p) + 2.0 * c * r;
            a[k] = p + s * w;
            a[k + 1] = q - s * w;
            b[k] = c * w - r;
            if (k + 1 < m) {
                z = s * b[k + 1];  // bulge at (k+2, k)
                b[k + 1] = c * b[k + 1];
                x = b[k];
            }
            for (double* rr : {rows.r0, rows.r1}) {
                if (!rr) continue;
                const double u = rr[k], v = rr[k + 1];
                rr[k] = c * u + s * v;
                rr[k + 1] = c * v - s * u;
            }
        }
    }
    // ascending order (selection: n <= kLeaf here or values only)
    if (rows.r0 || rows.r1) {
        for (int i = 0; i + 1 < n; ++i) {
            int k = i;
            for (int j = i + 1; j < n; ++j)
                if (a[j] < a[k]) k = j;
            if (k == i) continue;
            std::swap(a[i], a[k]);
            if (rows.r0) std::swap(rows.r0[i], rows.r0[k]);
            if (rows.r1) std::swap(rows.r1[i], rows.r1[k]);
        }
    } else {
        std::sort(a, a + n);
    }
    return status;
}

// ---------------------------------------------------------------------------
// Split tree of one unreduced block: balanced halving, merges levelled by
// height (both children of a merge finish before it runs).
// ---------------------------------------------------------------------------
struct Node {
    int64_t off;
    int nL, nR;
};
struct Tree {
    std::vector<std::pair<int64_t, int>> leaves;  // (off, size)
    std::vector<std::vector<Node>> levels;        // levels[h-1]: merges of height h
};

int build(Tree& t, int64_t off, int64_t size) {
    if (size <= kLeaf) {
        t.leaves.emplace_back(off, (int)size);
        return 0;
    }
    const int64_t nL = size / 2;
    const int h = std::max(build(t, off, nL), build(t, off + nL, size - nL)) + 1;
    if ((int)t.levels.size() < h) t.levels.resize(h);
    t.levels[h - 1].push_back(Node{off, (int)nL, (int)(size - nL)});
    return h;
}

// Workspace views (every array n long; a merge over [off, off + s) touches
// only that range).
struct Ws {
    double *lam, *blo, *bhi;          // node spectra and first/last eigenvector rows
    double *D, *Z, *RL, *RH;          // merged poles, z, parent first/last-row entries
    double *Dd, *RLd, *RHd;           // deflated columns (value, rows)
    double *tau, *zh, *PBL, *PBH;     // roots' offsets, Loewner z, parent rows of the roots
    double* W;                        // z^2 of the active poles
    int* org;                         // roots' origin poles
    int* st;                          // column state: 0 deflated, 1 active
};

// f(lambda) = 1 + rho sum_j z_j^2/(D_j - lambda) at lambda = D_o + tau, the
// denominators formed as (D_j - D_o) - tau: left (j <= kk) and right sums of
// the terms and of their derivatives, and the sum of |terms|.
struct Sums {
    double psi, dpsi, phi, dphi, abs;
};
Sums secular_sums(int K, const double* D, const double* W, int o, double tau, int kk) {
    Sums s{0.0, 0.0, 0.0, 0.0, 0.0};
    const double Do = D[o];
    for (int j = 0; j < K; ++j) {
        const double del = (D[j] - Do) - tau;
        const double t = W[j] / del;
        if (j <= kk) {
            s.psi += t;
            s.dpsi += t / del;
        } else {
            s.phi += t;
            s.dphi += t / del;
        }
        s.abs += fabs(t);
    }
    return s;
}

// Root k of 1 + rho sum z_j^2/(D_j - lambda) (strictly ascending D, nonzero
// z): bracket (D_k, D_k+1), or (D_(K-1), D_(K-1) + rho ||z||^2] for the last
// root.  Origin: the bracket end nearer to the root (sign of f at the
// midpoint).  Iteration: the two-pole rational model through the value and
// slope of f (each pole of the model absorbing the terms on its side, the
// "middle way"), solved for the new offset directly; bisection when the model
// root leaves the bracket.  Stops when |f| is within its rounding bound, the
// bracket has no double strictly inside, or a step is below an ulp.
int secular_root(int k, int K, const double* D, const double* W, double rho, double zz, int* org, double* tau_out) {
    if (K == 1) {
        *org = 0;
        *tau_out = rho * W[0];
        return 0;
    }
    int o, kk;
    double lo, hi, tau;
    if (k < K - 1) {
        kk = k;
        const double gap = D[k + 1] - D[k];
        const Sums s = secular_sums(K, D, W, k, 0.5 * gap, kk);
        const double f = 1.0 + rho * (s.psi + s.phi);
        if (f >= 0.0) {  // root left of the midpoint: origin D_k
            o = k;
            lo = 0.0;
            hi = 0.5 * gap;
        } else {
            o = k + 1;
            lo = -0.5 * gap;
            hi = 0.0;
        }
        tau = 0.5 * (lo + hi);
    } else {
        kk = K - 2;
        o = K - 1;
        lo = 0.0;
        hi = rho * zz * (1.0 + 8.0 * DBL_EPSILON) + DBL_MIN;
        tau = 0.5 * hi;
    }
    const double d1 = D[kk] - D[o], d2 = D[kk + 1] - D[o];  // model poles (offsets from D_o)
    for (int it = 1; it <= kSecCap; ++it) {
        const Sums s = secular_sums(K, D, W, o, tau, kk);
        const double f = 1.0 + rho * (s.psi + s.phi);
        if (fabs(f) <= 8.0 * DBL_EPSILON * (1.0 + rho * s.abs)) break;
        if (f < 0.0) lo = tau;
        else hi = tau;
        if (!(nextafter(lo, hi) < hi)) break;
        // model c + Q1/(d1 - x) + Q2/(d2 - x) through f and f' at tau
        const double e1 = d1 - tau, e2 = d2 - tau;
        const double Q1 = rho * s.dpsi * e1 * e1, Q2 = rho * s.dphi * e2 * e2;
        const double c = f - Q1 / e1 - Q2 / e2;
        // c (d1 - x)(d2 - x) + Q1 (d2 - x) + Q2 (d1 - x) = 0: c x^2 - B x + C = 0
        const double B = c * (d1 + d2) + Q1 + Q2;
        const double C = c * d1 * d2 + Q1 * d2 + Q2 * d1;
        double disc = B * B - 4.0 * c * C;
        disc = disc > 0.0 ? sqrt(disc) : 0.0;
        const double qq = (B >= 0.0) ? B + disc : B - disc;
        double x1 = (c != 0.0) ? qq / (2.0 * c) : NAN;
        double x2 = (qq != 0.0) ? 2.0 * C / qq : NAN;
        const bool in1 = x1 > lo && x1 < hi, in2 = x2 > lo && x2 < hi;
        double tn;
        if (in1 && in2) tn = fabs(x1 - tau) < fabs(x2 - tau) ? x1 : x2;
        else if (in1) tn = x1;
        else if (in2) tn = x2;
        else tn = 0.5 * (lo + hi);
        const bool small = fabs(tn - tau) <= 2.0 * DBL_EPSILON * fabs(tau);
        tau = tn;
        if (small) break;
        if (it == kSecCap) {
            *org = o;
            *tau_out = tau;
            return 1;
        }
    }
    *org = o;
    *tau_out = tau;
    return 0;
}

// One merge over [off, off + s) with left child size nL and coupling beta;
// top = the block's root merge (eigenvalues only).  par: parallelise the
// per-root and per-pole loops (levels with fewer merges than threads).
int merge(const Ws& w, int64_t off, int nL, int nR, double beta, bool top, bool par, int nth) {
    const int s = nL + nR;
    const double rho = 2.0 * fabs(beta);
    const double sg = (beta < 0.0) ? -1.0 : 1.0;
    const double r2 = 1.0 / sqrt(2.0);
    double* lam = w.lam + off;
    double* D = w.D + off;
    double* Z = w.Z + off;
    double* RL = w.RL + off;
    double* RH = w.RH + off;
    // merge of the two ascending child spectra (ties: left first), z and
    // the parent's outer rows alongside
    {
        int i = 0, j = nL, t = 0;
        while (i < nL || j < s) {
            const bool left = (j >= s) || (i < nL && lam[i] <= lam[j]);
            const int c = left ? i++ : j++;
            D[t] = lam[c];
            if (left) {
                Z[t] = w.bhi[off + c] * r2;
                RL[t] = w.blo[off + c];
                RH[t] = 0.0;
            } else {
                Z[t] = sg * w.blo[off + c] * r2;
                RL[t] = 0.0;
                RH[t] = w.bhi[off + c];
            }
            ++t;
        }
    }
    // deflation (tolerance 8 eps max(max|D|, 1) on the scaled block):
    // negligible z, then close consecutive poles rotated together
    const double tol = 8.0 * DBL_EPSILON * std::max(std::max(fabs(D[0]), fabs(D[s - 1])), 1.0);
    int* st = w.st + off;
    int p = -1;
    for (int j = 0; j < s; ++j) {
        if (rho * fabs(Z[j]) <= tol) {
            st[j] = 0;
            continue;
        }
        st[j] = 1;
        if (p >= 0) {
            const double t = hypot(Z[p], Z[j]);
            const double c = Z[j] / t, sn = Z[p] / t;
            if (fabs((D[j] - D[p]) * c * sn) <= tol) {
                // G = [c -s; s c] on (p, j): z_p -> 0, z_j -> t; p deflates
                const double dp = c * c * D[p] + sn * sn * D[j];
                const double dj = sn * sn * D[p] + c * c * D[j];
                const double lo = D[p], hi = D[j];
                D[p] = std::min(std::max(dp, lo), hi);
                D[j] = std::min(std::max(dj, lo), hi);
                Z[p] = 0.0;
                Z[j] = t;
                for (double* R : {RL, RH}) {
                    const double u = R[p], v = R[j];
                    R[p] = c * u - sn * v;
                    R[j] = sn * u + c * v;
                }
                st[p] = 0;
            }
        }
        p = j;
    }
    // compaction: active columns to the front of D, Z, RL, RH; deflated ones
    // (value and rows) to Dd, RLd, RHd, sorted by value
    int K = 0, nd = 0;
    double* Dd = w.Dd + off;
    double* RLd = w.RLd + off;
    double* RHd = w.RHd + off;
    for (int j = 0; j < s; ++j) {
        if (st[j]) {
            D[K] = D[j];
            Z[K] = Z[j];
            RL[K] = RL[j];
            RH[K] = RH[j];
            ++K;
        } else {
            Dd[nd] = D[j];
            RLd[nd] = RL[j];
            RHd[nd] = RH[j];
            ++nd;
        }
    }
    {
        // the rotations can leave the deflated values out of order: sort
        // them with their rows (an index sort through the tau slice, free here)
        bool sorted = true;
        for (int q = 1; q < nd; ++q)
            if (Dd[q] < Dd[q - 1]) sorted = false;
        if (!sorted) {
            std::vector<int> idx(nd);
            for (int q = 0; q < nd; ++q) idx[q] = q;
            std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return Dd[x] < Dd[y]; });
            double* tmp = w.tau + off;
            for (double* A : {Dd, RLd, RHd}) {
                for (int q = 0; q < nd; ++q) tmp[q] = A[idx[q]];
                memcpy(A, tmp, sizeof(double) * nd);
            }
        }
    }
    double* Wz = w.W + off;
    double zz = 0.0;
    for (int i = 0; i < K; ++i) {
        Wz[i] = Z[i] * Z[i];
        zz += Wz[i];
    }
    // secular roots
    int* org = w.org + off;
    double* tau = w.tau + off;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad) if (par) num_threads(nth)
    for (int k = 0; k < K; ++k) bad |= secular_root(k, K, D, Wz, rho, zz, &org[k], &tau[k]);
    double* PBL = w.PBL + off;
    double* PBH = w.PBH + off;
    if (!top) {
        // Loewner z: zhat_i^2 = prod_k (lambda_k - D_i) / (rho prod_(j != i) (D_j - D_i)),
        // as a chain of ratios of like-signed factors, the sign of z_i
        double* zh = w.zh + off;
#pragma omp parallel for schedule(static) if (par) num_threads(nth)
        for (int i = 0; i < K; ++i) {
            double prod = 1.0 / rho;
            for (int k = 0; k < K; ++k) {
                const double num = (D[org[k]] - D[i]) + tau[k];
                const double den = (k < i) ? D[k] - D[i] : (k < K - 1 ? D[k + 1] - D[i] : 1.0);
                prod *= num / den;
            }
            const double zi = sqrt(std::max(prod, 0.0));
            zh[i] = (Z[i] < 0.0) ? -zi : zi;
        }
        // parent rows of every root: two dot products with the unit secular
        // vector y_k(i) = zhat_i / (D_i - lambda_k), streamed
#pragma omp parallel for schedule(static) if (par) num_threads(nth)
        for (int k = 0; k < K; ++k) {
            const double Do = D[org[k]], tk = tau[k];
            double ss = 0.0, bl = 0.0, bh = 0.0;
            for (int i = 0; i < K; ++i) {
                const double y = zh[i] / ((D[i] - Do) - tk);
                ss += y * y;
                bl += RL[i] * y;
                bh += RH[i] * y;
            }
            const double inv = 1.0 / sqrt(ss);
            PBL[k] = bl * inv;
            PBH[k] = bh * inv;
        }
    }
    // assembly: the parent's spectrum (roots and deflated values, ascending)
    // and rows; the roots are read before lam is overwritten (tau, org, D
    // live in other arrays)
    {
        int k = 0, q = 0;
        for (int t = 0; t < s; ++t) {
            const double lr = (k < K) ? D[org[k]] + tau[k] : INFINITY;
            const bool root = (k < K) && (q >= nd || lr <= Dd[q]);
            if (root) {
                lam[t] = lr;
                if (!top) {
                    w.blo[off + t] = PBL[k];
                    w.bhi[off + t] = PBH[k];
                }
                ++k;
            } else {
                lam[t] = Dd[q];
                if (!top) {
                    w.blo[off + t] = RLd[q];
                    w.bhi[off + t] = RHd[q];
                }
                ++q;
            }
        }
    }
    return bad;
}

int nthreads_of(int want) {
#ifdef _OPENMP
    return want > 0 ? want : omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

// One unreduced block [0, n) of (d, e), already scaled: eigenvalues into lam.
int solve_block(int64_t n, const double* d, const double* e, const Ws& w, int nth) {
    if (n <= kLeaf) {
        double b[kLeaf];
        for (int64_t i = 0; i < n; ++i) w.lam[i] = d[i];
        for (int64_t i = 0; i + 1 < n; ++i) b[i] = e[i];
        return qr_solve((int)n, w.lam, b, QrRows{nullptr, nullptr});
    }
    Tree t;
    build(t, 0, n);
    int bad = 0;
    // leaves: torn diagonal (every leaf boundary is a tear), QR with the
    // first and last eigenvector rows
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad) num_threads(nth)
    for (size_t li = 0; li < t.leaves.size(); ++li) {
        const int64_t off = t.leaves[li].first;
        const int sz = t.leaves[li].second;
        double b[kLeaf];
        double* a = w.lam + off;
        for (int i = 0; i < sz; ++i) a[i] = d[off + i];
        for (int i = 0; i + 1 < sz; ++i) b[i] = e[off + i];
        if (off > 0) a[0] -= fabs(e[off - 1]);
        if (off + sz < n) a[sz - 1] -= fabs(e[off + sz - 1]);
        bad |= qr_solve(sz, a, b, QrRows{w.blo + off, w.bhi + off});
    }
    for (size_t h = 0; h < t.levels.size(); ++h) {
        const std::vector<Node>& L = t.levels[h];
        const bool top = (h + 1 == t.levels.size());
        if ((int)L.size() >= nth) {
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad) num_threads(nth)
            for (size_t m = 0; m < L.size(); ++m)
                bad |= merge(w, L[m].off, L[m].nL, L[m].nR, e[L[m].off + L[m].nL - 1], top && L.size() == 1, false, nth);
        } else {
            for (size_t m = 0; m < L.size(); ++m)
                bad |= merge(w, L[m].off, L[m].nL, L[m].nR, e[L[m].off + L[m].nL - 1], top && L.size() == 1, true, nth);
        }
    }
    return bad;
}

}  // namespace

extern "C" {

int tde_host_workspace(int64_t n, int64_t* lwork, int64_t* liwork) {
    if (n < 0 || !lwork || !liwork) return TDE_HOST_EINVAL;
    *lwork = 16 * n;
    *liwork = 2 * n;
    return TDE_HOST_OK;
}

int tde_host_eigvals(const double* d, const double* e, int64_t n, double* lambda, double* work, int64_t lwork,
                     int* iwork, int64_t liwork, int nthreads) {
    if (n < 0) return TDE_HOST_EINVAL;
    if (n == 0) return TDE_HOST_OK;
    if (!d || !lambda || (n > 1 && !e) || !work || !iwork || lwork < 16 * n || liwork < 2 * n || nthreads < 0)
        return TDE_HOST_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(d[i]) || (i + 1 < n && !isfinite(e[i]))) return TDE_HOST_ENONFINITE;
    const int nth = nthreads_of(nthreads);
    // workspace: lam, blo, bhi, D, Z, RL, RH, Dd, RLd, RHd, tau, zh, PBL, PBH, W,
    // and the scaled copy of d (15 + 1 arrays of n doubles); org, st (2 n ints)
    double* base = work;
    Ws w;
    double** dbl[] = {&w.lam, &w.blo, &w.bhi, &w.D, &w.Z, &w.RL, &w.RH, &w.Dd, &w.RLd, &w.RHd,
                      &w.tau, &w.zh, &w.PBL, &w.PBH, &w.W};
    for (int a = 0; a < 15; ++a) *dbl[a] = base + a * n;
    double* ds = base + 15 * n;  // scaled diagonal of the current block
    w.org = iwork;
    w.st = iwork + n;
    int status = TDE_HOST_OK;
    int64_t b0 = 0;
    while (b0 < n) {
        // unreduced block [b0, b1): couplings with |e_i| <= eps sqrt|d_i| sqrt|d_(i+1)| are dropped
        int64_t b1 = b0 + 1;
        while (b1 < n && fabs(e[b1 - 1]) > DBL_EPSILON * sqrt(fabs(d[b1 - 1])) * sqrt(fabs(d[b1]))) ++b1;
        const int64_t m = b1 - b0;
        if (m == 1) {
            lambda[b0] = d[b0];
        } else {
            // exact power-of-two scale of the block: max |T_ij| in [1/2, 1)
            double mx = 0.0;
            for (int64_t i = b0; i < b1; ++i) mx = std::max(mx, fabs(d[i]));
            for (int64_t i = b0; i + 1 < b1; ++i) mx = std::max(mx, fabs(e[i]));
            int ex = 0;
            if (mx > 0.0) frexp(mx, &ex);
            // the block's scaled couplings live in its slice of lambda, which
            // receives the block's eigenvalues only after its solve
            double* es = lambda + b0;
            for (int64_t i = 0; i < m; ++i) ds[i] = ldexp(d[b0 + i], -ex);
            for (int64_t i = 0; i + 1 < m; ++i) es[i] = ldexp(e[b0 + i], -ex);
            const Ws wb = w;  // the block uses the leading m entries of every array
            const int bad = solve_block(m, ds, es, wb, nth);
            if (bad) status = TDE_HOST_ENOCONV;
            for (int64_t i = 0; i < m; ++i) lambda[b0 + i] = ldexp(w.lam[i], ex);
        }
        b0 = b1;
    }
    std::sort(lambda, lambda + n);
    return status;
}

}  // extern "C"
