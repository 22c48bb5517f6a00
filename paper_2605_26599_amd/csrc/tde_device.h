// Per-thread bodies of the BR D&C kernels (gfx950).  Every element-parallel
// kernel in tde_kernels.hip is a thin wrapper that maps its thread index to one
// call of a body below; the bodies hold all of the method's arithmetic.
//
// Notation follows the paper (Section 3.1, merge problem): a merge of children
// L and R has poles D = Lambda_L (+) Lambda_R, secular vector
// z = concat(bhi(Q_L), blo(Q_R)) and coupling rho; the parent eigenvalues are
// the roots of 1 + rho * sum_j z_j^2 / (D_j - lambda) = 0.  We use the
// normalised tear z~ = z / sqrt(2), rho~ = 2 |beta| (beta the torn
// off-diagonal), sign(beta) applied to the right half, so that ||z~|| = 1.
#pragma once
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "tde_internal.h"

#ifndef TDE_DEV
#define TDE_DEV __device__ __forceinline__
#endif
#ifndef TDE_ATOMIC_MAX_U64
#define TDE_ATOMIC_MAX_U64(p, v) atomicMax((p), (v))
#endif
#ifndef TDE_ATOMIC_OR
#define TDE_ATOMIC_OR(p, v) atomicOr((p), (v))
#endif
// Hardware reciprocal estimate (refined by rcp_nr below).
#ifndef TDE_RCP_ESTIMATE
#define TDE_RCP_ESTIMATE(x) __builtin_amdgcn_rcp(x)
#endif
// Hardware reciprocal square root estimate (refined by rot_gen below).
#ifndef TDE_RSQ_ESTIMATE
#define TDE_RSQ_ESTIMATE(x) __builtin_amdgcn_rsq(x)
#endif

namespace tde {

// 1/x from the hardware estimate and two Newton steps (each squares the
// relative error), about an ulp: the sweeps' per-term division.
TDE_DEV double rcp_nr(double x) {
    double y = TDE_RCP_ESTIMATE(x);
    double t = fma(-x, y, 1.0);
    y = fma(y, t, y);
    t = fma(-x, y, 1.0);
    return fma(y, t, y);
}

TDE_DEV unsigned long long dbits(double x) {
    union { double d; unsigned long long u; } c;
    c.d = x;
    return c.u;
}
TDE_DEV double bitsd(unsigned long long u) {
    union { double d; unsigned long long u; } c;
    c.u = u;
    return c.d;
}

// Exact power-of-two scale 2^ceil(log2 max|T_ij|) of a problem (driver-level
// scaling of unreduced blocks, Section 4.2); 1 for the zero matrix.
TDE_DEV double scale_of(unsigned long long maxbits) {
    double mx = bitsd(maxbits);
    if (!(mx > 0.0) || !(mx <= DBL_MAX)) return 1.0;
    int ex;
    frexp(mx, &ex);
    return ldexp(1.0, ex);
}

// Largest m in [lo, hi] with mr[m].pk <= t (merge lookup within a range known
// to contain the answer).
TDE_DEV int find_merge_in(const MergeRec* __restrict__ mr, int lo, int hi, long long t) {
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (mr[mid].pk <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Largest m in [0, M) with key(m) <= t, for nondecreasing keys (merge lookup).
TDE_DEV int find_merge(const MergeRec* __restrict__ mr, int M, long long t) {
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (mr[mid].pk <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Coupling of a merge: rho~ = 2|beta| / scale and sign(beta), beta the torn
// off-diagonal e[off + nL - 1] (paper Eq. dc-split; tearing convention of DESIGN).
TDE_DEV double merge_rho(const MergeRec& R, const double* __restrict__ e,
                         const unsigned long long* __restrict__ pmax, double* sgn) {
    double beta = e[R.off + R.nL - 1] * (1.0 / scale_of(pmax[R.prob]));
    *sgn = (beta < 0.0) ? -1.0 : 1.0;
    return 2.0 * fabs(beta);
}

// Deflation tolerance of a merge: 8 eps max(max|D|, 1).  The usual
// 8 eps max(max|D|, max|z~|) with max|z~| replaced by its bound ||z~|| = 1, so
// the test needs no reduction over the merge.  The poles are sorted, so
// max|D| is attained at an end.
TDE_DEV double merge_tol(const double* __restrict__ D, long long pk, int s) {
    const double dmax = fmax(fabs(D[pk]), fabs(D[pk + s - 1]));
    return 8.0 * DBL_EPSILON * fmax(dmax, 1.0);
}

// Close-pole test for consecutive poles a < b (Section 4.1, deflation): the
// Givens rotation that zeroes z_a drops an off-diagonal (D_b - D_a) c s.
TDE_DEV bool close_pair(double Da, double za, double Db, double zb, double tol) {
#pragma clang fp contract(off)
    double t = hypot(za, zb);
    double c = zb / t, s = za / t;
    return fabs((Db - Da) * c * s) <= tol;
}

// ---------------------------------------------------------------------------
// Leaf: implicit QL with a Wilkinson shift on one small tridiagonal,
// accumulating only selected rows of the eigenvector matrix (Algorithm 1,
// leaf step; rows of Q G are the selected rows of Q times G, Lemma 2).
//
// The step is the implicit symmetric QR step with a Wilkinson shift of Golub
// and Van Loan (Matrix Computations, 4th ed., Section 8.3, Algorithm 8.3.2)
// in its QL mirror image: shift from the top 2x2 block of the active block
// [l, m], first plane rotation from the shifted last column, bulge chased
// upward, top coupling converging.  A rotation in plane (k, k+1) with cosine c
// and sine s maps rows k, k+1 to c r_k - s r_(k+1), s r_k + c r_(k+1); applied
// from both sides it changes the 2x2 block (a, f; f, g) through
// w = s (a - g) + 2 c f:  a' = a - s w,  g' = g + s w,  f' = c w - f
// (the rotation's c^2 / s^2 form rewritten with c^2 + s^2 = 1, trace kept
// exactly), scales the coupling above by c and leaves the bulge s e_(k-1) at
// (k-1, k+1); the next rotation (c, s) = (e_(k+1), b)/hypot(b, e_(k+1))
// removes a bulge b at (k, k+2).  The eigenvector rows follow Q <- Q R^T.
//
// `rows` applies each plane rotation to columns k, k+1 of the tracked rows
// (rot) and mirrors the final ascending sort (swap).  The scalar recurrence is
// the same for every choice of tracked rows, and contraction is off, so the
// forward pass (rows 0 and l-1) and the adjoint's recomputation (one row per
// lane) see bitwise the same eigenvalues and rotations.  Arrays are strided
// (st = lanes sharing an LDS tile).  Returns 0 or ST_LEAF_NOCONV (an
// eigenvalue needed more than 60 steps).
// ---------------------------------------------------------------------------
// Plane rotation (c, s) with c = x/r, s = y/r, r = sqrt(x^2 + y^2) (c = 1,
// s = 0 when r = 0).  In the usual range r comes from one reciprocal square
// root (hardware estimate and two Newton steps) instead of a scaled hypot
// and two divisions; outside it (squares that could underflow or overflow)
// the scaled hypot and the divisions are used.
TDE_DEV double rot_gen(double x, double y, double* c, double* s) {
#pragma clang fp contract(off)
    const double mx = fmax(fabs(x), fabs(y));
    if (mx > 1e-140 && mx < 1e140) {
        const double r2 = x * x + y * y;
        double q = TDE_RSQ_ESTIMATE(r2);
        q = q * (1.5 - (0.5 * r2) * (q * q));
        q = q * (1.5 - (0.5 * r2) * (q * q));
        *c = x * q;
        *s = y * q;
        return r2 * q;
    }
    const double r = hypot(x, y);
    *c = (r == 0.0) ? 1.0 : x / r;
    *s = (r == 0.0) ? 0.0 : y / r;
    return r;
}

template <class Rows>
TDE_DEV int leaf_ql_core(int nl, double* d, double* e, int st, Rows& rows, unsigned* nrot) {
#pragma clang fp contract(off)
#define A_(p, i) p[(i) * st]
    int status = 0;
    unsigned nr = 0;
    A_(e, nl - 1) = 0.0;
    for (int l = 0; l < nl; ++l) {
        int steps = 0;
        for (;;) {
            // end of the unreduced block that starts at l (the entries are
            // read four at a time, so the loads do not wait on each other)
            int m = l;
            for (;;) {
                if (m + 4 < nl) {
                    const double e0 = A_(e, m), e1 = A_(e, m + 1), e2 = A_(e, m + 2), e3 = A_(e, m + 3);
                    const double d0 = A_(d, m), d1 = A_(d, m + 1), d2 = A_(d, m + 2), d3 = A_(d, m + 3),
                                 d4 = A_(d, m + 4);
                    if (!(fabs(e0) > DBL_EPSILON * (fabs(d0) + fabs(d1)))) break;
                    if (!(fabs(e1) > DBL_EPSILON * (fabs(d1) + fabs(d2)))) { m += 1; break; }
                    if (!(fabs(e2) > DBL_EPSILON * (fabs(d2) + fabs(d3)))) { m += 2; break; }
                    if (!(fabs(e3) > DBL_EPSILON * (fabs(d3) + fabs(d4)))) { m += 3; break; }
                    m += 4;
                } else {
                    while (m + 1 < nl && fabs(A_(e, m)) > DBL_EPSILON * (fabs(A_(d, m)) + fabs(A_(d, m + 1)))) ++m;
                    break;
                }
            }
            if (m + 1 < nl) A_(e, m) = 0.0;
            if (m == l) break;  // d[l] converged
            if (++steps > 60) {
                status = ST_LEAF_NOCONV;
                break;
            }
            // Wilkinson shift: eigenvalue of the top 2x2 block nearer to d[l]
            double mu = A_(d, l);
            {
                const double f = A_(e, l);
                const double h = (A_(d, l + 1) - mu) / (2.0 * f);
                const double r = hypot(h, 1.0);
                mu -= f / (h + (h >= 0.0 ? r : -r));
            }
            double c, s;
            (void)rot_gen(A_(d, m) - mu, A_(e, m - 1), &c, &s);
            // the chase carries the entries it has just updated in registers
            // and loads the next two untouched ones ahead (d(k-1), e(k-2):
            // nothing writes them before their use), so no step waits on a
            // store-then-load through LDS
            double bulge = 0.0;
            double ek1 = 0.0;            // e(k+1) as updated by the previous step
            double dk1 = A_(d, m);       // d(k+1)
            double ek = A_(e, m - 1);    // e(k)
            double dk = A_(d, m - 1);    // d(k)
            double ekm1 = (m - 2 >= l) ? A_(e, m - 2) : 0.0;  // e(k-1)
            rows.chase_begin(m);
            for (int k = m - 1; k >= l; --k) {
                const double dn = (k - 1 >= l) ? A_(d, k - 1) : 0.0;
                const double en = (k - 2 >= l) ? A_(e, k - 2) : 0.0;
                if (k < m - 1) A_(e, k + 1) = rot_gen(ek1, bulge, &c, &s);
                const double a = dk, g = dk1, f = ek;
                const double w = s * (a - g) + 2.0 * c * f;
                const double dkn = a - s * w;
                A_(d, k) = dkn;
                A_(d, k + 1) = g + s * w;
                const double ekn = c * w - f;
                A_(e, k) = ekn;
                double ekm1n = ekm1;
                if (k > l) {
                    bulge = s * ekm1;
                    ekm1n = c * ekm1;
                    A_(e, k - 1) = ekm1n;
                }
                ++nr;
                rows.rot(k, c, s);
                ek1 = ekn;
                dk1 = dkn;
                ek = ekm1n;
                dk = dn;
                ekm1 = en;
            }
            rows.chase_end(l);
        }
    }
    // ascending order, rows permuted alongside
    for (int i = 0; i + 1 < nl; ++i) {
        int k = i;
        double v = A_(d, i);
        for (int j = i + 1; j < nl; ++j)
            if (A_(d, j) < v) { k = j; v = A_(d, j); }
        if (k != i) {
            A_(d, k) = A_(d, i);
            A_(d, i) = v;
            rows.swap(i, k);
        }
    }
    *nrot = nr;
    return status;
#undef A_
}

// One tracked row q (row `row` of Q; q starts as that row of the identity).
// A chase applies rot(k) for k = m-1 down to l; the entry it is about to
// combine with (q[k+1]) is carried in a register from one rotation to the
// next (chase_begin loads q[m], chase_end stores the last one at q[l]), so
// no rotation waits on the previous one's store.
struct RowTrack {
    double* q;
    int st;
    double cur;
    TDE_DEV void init(int nl, int row) {
        for (int i = 0; i < nl; ++i) q[i * st] = (i == row) ? 1.0 : 0.0;
    }
    TDE_DEV void chase_begin(int m) { cur = q[m * st]; }
    TDE_DEV void chase_end(int l) { q[l * st] = cur; }
    TDE_DEV void rot(int i, double c, double s) {
#pragma clang fp contract(off)
        const double t = cur;
        const double qi = q[i * st];
        q[(i + 1) * st] = s * qi + c * t;
        cur = c * qi - s * t;
    }
    TDE_DEV void swap(int i, int k) {
        const double t = q[i * st];
        q[i * st] = q[k * st];
        q[k * st] = t;
    }
};

struct TwoRows {
    RowTrack a, b;
    TDE_DEV void chase_begin(int m) {
        a.chase_begin(m);
        b.chase_begin(m);
    }
    TDE_DEV void chase_end(int l) {
        a.chase_end(l);
        b.chase_end(l);
    }
    TDE_DEV void rot(int i, double c, double s) {
        a.rot(i, c, s);
        b.rot(i, c, s);
    }
    TDE_DEV void swap(int i, int k) {
        a.swap(i, k);
        b.swap(i, k);
    }
};

// Forward leaf: eigenvalues (ascending, in d) and rows ra and rb (r0, r1;
// by default 0 and l-1, the boundary rows).
TDE_DEV int leaf_ql(int nl, double* d, double* e, double* r0, double* r1, int st, unsigned* nrot, int ra,
                    int rb) {
    TwoRows rows;
    rows.a.q = r0;
    rows.a.st = st;
    rows.b.q = r1;
    rows.b.st = st;
    rows.a.init(nl, ra);
    rows.b.init(nl, rb);
    return leaf_ql_core(nl, d, e, st, rows, nrot);
}

// ---------------------------------------------------------------------------
// Secular equation (Section 2.2, the rank-one merge; Section 4.1 root solve;
// compact roots as in the appendix on compact delta reconstruction).
// Root k (0-based) of f(lambda) = 1 + rho sum_j z_j^2/(D_j - lambda) for
// strictly ascending poles D[0..K) and nonzero z.  Output: origin pole index
// org in {k, k+1} and offset tau with lambda_k = D[org] + tau; every
// denominator is formed as (D_j - D_org) - tau, so the near-pole ones carry
// no cancellation.
//
// Each step fits a rational model
//     g(x) = c + q/(d1 - x) + Q/(d2 - x),   d1 = D_kk - D_org, d2 = D_kk+1 - D_org,
// to the value and slope of f at the current offset and takes its root in the
// bracket as the next offset x (solved for x directly, not as a correction,
// which would cancel when the root sits next to its pole).  Two fits are used:
//  - fixed weight: the origin pole keeps its exact weight rho z_org^2 and the
//    other model pole absorbs the slope of every other term;
//  - middle way: each model pole absorbs the slope of all poles on its side.
// Fixed weight is used first; if an iteration fails to cut |f| tenfold the
// root switches to the middle way for good.  Safeguard: bisection of the
// bracket.  The interior roots start from the bracket midpoint, which also
// picks the nearer pole as origin; the last root starts from the root of the
// equation truncated to its two nearest poles (a lower bound).
// Stops when |f| is within its rounding-error bound, when a step moves tau by
// less than an ulp, or when the bracket cannot shrink.  Returns the number of
// sweeps after the first, negative if the cap was hit.
// ---------------------------------------------------------------------------
TDE_DEV double model_root(double f, double tau, double d1, double d2, double q, double Q, double lo,
                          double hi) {
    // c(d1-x)(d2-x) + q(d2-x) + Q(d1-x) = 0  <=>  c x^2 - A x + C0 = 0
    const double c = f - q * rcp_nr(d1 - tau) - Q * rcp_nr(d2 - tau);
    const double A = c * (d1 + d2) + q + Q;
    const double C0 = c * d1 * d2 + q * d2 + Q * d1;
    double disc = A * A - 4.0 * C0 * c;
    if (!(disc >= 0.0)) disc = 0.0;
    const double sq = sqrt(disc);
    const double den = (A >= 0.0) ? A + sq : A - sq;
    const double r1 = (c != 0.0) ? den * rcp_nr(2.0 * c) : NAN;
    const double r2 = (den != 0.0) ? 2.0 * C0 * rcp_nr(den) : NAN;
    const bool in1 = r1 > lo && r1 < hi;
    const bool in2 = r2 > lo && r2 < hi;
    if (in1 && in2) return 0.5 * (r1 + r2);
    if (in2) return r2;
    if (in1) return r1;
    return 0.5 * (lo + hi);
}

// Sweeps over the poles are split across a group of G lanes (lane `sub` takes
// poles sub, sub+G, ...); Red::sum returns the group total, bitwise identical
// in every lane of the group, so all lanes take the same branches.
struct RedSerial {
    TDE_DEV static double sum(double x) { return x; }
    TDE_DEV static double prod(double x) { return x; }
};

// State of one secular root between pole sweeps.
struct SecRoot {
    int o;                // origin pole
    double lo, hi, tau;   // bracket and current offset from D_o
    double d1, d2;        // the bracketing poles D_kk, D_kk+1 relative to D_o
    double zo, wo;        // z_o and the origin weight rho z_o^2
    double fprev;
    bool orgl;            // origin is the left bracketing pole
    bool fixed_weight;
};

// Interior root k < K-1 (kk = k): from the sums at the bracket midpoint with
// origin kk (ps, dps over j < kk; ph, dph over j > kk+1) pick the nearer pole
// as origin and take the first model step.  Returns true when the midpoint is
// the root itself (r->tau final).
TDE_DEV bool sec_start_interior(int k, const double* __restrict__ D, const double* __restrict__ Z, double rho,
                                double ps, double dps, double ph, double dph, SecRoot* r) {
    const int kk = k;
    const double dk = D[kk], dk1 = D[kk + 1];
    const double mid = 0.5 * (dk1 - dk);
    const double ak = Z[kk] / (-mid), ak1 = Z[kk + 1] / mid;
    const double f = 1.0 + rho * (ps + ph + Z[kk] * ak + Z[kk + 1] * ak1);
    if (f >= 0.0) { r->o = k; r->lo = 0.0; r->hi = mid; r->tau = mid; }
    else { r->o = k + 1; r->lo = -mid; r->hi = 0.0; r->tau = -mid; }
    const double Do = D[r->o];
    r->d1 = dk - Do;
    r->d2 = dk1 - Do;
    r->zo = Z[r->o];
    r->wo = rho * r->zo * r->zo;
    r->orgl = (r->o == kk);
    r->fixed_weight = true;
    r->fprev = INFINITY;
    if (f == 0.0) return true;
    double q, Q;
    if (r->orgl) { q = r->wo; Q = (r->d2 - r->tau) * (r->d2 - r->tau) * rho * (dps + dph + ak1 * ak1); }
    else { Q = r->wo; q = (r->d1 - r->tau) * (r->d1 - r->tau) * rho * (dps + dph + ak * ak); }
    r->tau = model_root(f, r->tau, r->d1, r->d2, q, Q, r->lo, r->hi);
    return false;
}

// Last root (k = K-1, origin K-1): bracket (0, rho ||z||^2] and the first
// offset from the equation truncated to the two nearest poles (a lower bound).
TDE_DEV void sec_start_last(int K, const double* __restrict__ D, const double* __restrict__ Z, double rho, double zz,
                            SecRoot* r) {
    const double dk = D[K - 2], dk1 = D[K - 1];
    r->o = K - 1;
    r->lo = 0.0;
    r->hi = rho * zz * (1.0 + 4.0 * DBL_EPSILON) + DBL_MIN;
    const double w1 = rho * Z[K - 1] * Z[K - 1], w2 = rho * Z[K - 2] * Z[K - 2], g = dk1 - dk;
    const double b = g - w1 - w2, sq = sqrt(b * b + 4.0 * w1 * g);
    const double t2 = (b <= 0.0) ? 0.5 * (sq - b) : 2.0 * w1 * g / (b + sq);
    r->tau = (t2 > r->lo && t2 < r->hi) ? t2 : 0.5 * r->hi;
    r->d1 = dk - dk1;
    r->d2 = 0.0;
    r->zo = Z[K - 1];
    r->wo = rho * r->zo * r->zo;
    r->orgl = false;
    r->fixed_weight = true;
    r->fprev = INFINITY;
}

// One iteration from a sweep at r->tau: psi, dpsi over the poles j <= kk and
// phi, dphi over j > kk (the origin excluded from both), err = sum of |terms|
// over those poles.  Returns 1 when converged (r->tau final), else 0 with the
// next offset in r->tau.
TDE_DEV int sec_update(SecRoot* r, double rho, double psi, double dpsi, double phi, double dphi, double err) {
    const double tau = r->tau;
    const double to = -r->zo * rcp_nr(tau);
    const double termo = r->zo * to, dto = to * to;
    const double f = 1.0 + rho * (psi + phi + termo);
    err += fabs(termo);
    if (fabs(f) <= 8.0 * DBL_EPSILON * (1.0 + rho * err)) return 1;
    if (f < 0.0) r->lo = tau;
    else r->hi = tau;
    if (r->hi - r->lo <= 2.0 * DBL_EPSILON * fmax(fabs(r->lo), fabs(r->hi))) return 1;
    if (r->fixed_weight && fabs(f) > 0.1 * fabs(r->fprev)) r->fixed_weight = false;
    r->fprev = f;
    double q, Q;
    const double d1 = r->d1, d2 = r->d2;
    if (r->fixed_weight) {
        if (r->orgl) { q = r->wo; Q = (d2 - tau) * (d2 - tau) * rho * (dpsi + dphi); }
        else { Q = r->wo; q = (d1 - tau) * (d1 - tau) * rho * (dpsi + dphi); }
    } else {
        q = (d1 - tau) * (d1 - tau) * rho * (dpsi + (r->orgl ? dto : 0.0));
        Q = (d2 - tau) * (d2 - tau) * rho * (dphi + (r->orgl ? 0.0 : dto));
    }
    const double tn = model_root(f, tau, d1, d2, q, Q, r->lo, r->hi);
    r->tau = tn;
    if (fabs(tn - tau) <= 2.0 * DBL_EPSILON * fabs(tau)) return 1;
    return 0;
}

// One pole sweep for a root at offset tau from pole Do: left poles j < L1 and
// right poles j >= R0 (those in [L1, R0) are excluded); lane `sub` of a
// group of G takes j = sub, sub + G, ...  Per pole term: r = 1/((D_j - Do) -
// tau), t = w_j r, t r.  s[0..3] receive the group totals psi, dpsi, phi,
// dphi and, with ZZ, s[4] the sum of the weights w_j = z_j^2.
// The root lies strictly between the poles L1 - 1 and R0 (its offset never
// reaches a bracketing pole, and a difference of distinct doubles is never
// 0), so every left term is <= 0 and every right term >= 0: the split is
// taken by sign (min / max) rather than by index.
template <class Red, bool ZZ>
TDE_DEV void sec_sweep(int K, const double* __restrict__ D, const double* __restrict__ W, double Do, double tau,
                       int L1, int R0, int sub, int G, double* s) {
    double ps = 0.0, dps = 0.0, ph = 0.0, dph = 0.0, zz = 0.0;
    const unsigned exw = (unsigned)(R0 - L1);
    auto term = [&](int j, double dj, double wr) {
        const double rr = rcp_nr((dj - Do) - tau);
        const double wj = ((unsigned)(j - L1) < exw) ? 0.0 : wr;
        const double t = wj * rr;
        const double tl = fmin(t, 0.0), th = fmax(t, 0.0);
        ps += tl;
        dps = fma(tl, rr, dps);
        ph += th;
        dph = fma(th, rr, dph);
        if (ZZ) zz += wr;
    };
    int j = sub;
    // four terms per step; the next step's poles and weights are loaded
    // before this step's terms are evaluated, so the loads overlap the math
    if (j + 3 * G < K) {
        double a0 = D[j], a1 = D[j + G], a2 = D[j + 2 * G], a3 = D[j + 3 * G];
        double b0 = W[j], b1 = W[j + G], b2 = W[j + 2 * G], b3 = W[j + 3 * G];
        for (;;) {
            const int jn = j + 4 * G;
            const bool more = jn + 3 * G < K;
            double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0, e3 = 0.0;
            if (more) {
                c0 = D[jn];
                c1 = D[jn + G];
                c2 = D[jn + 2 * G];
                c3 = D[jn + 3 * G];
                e0 = W[jn];
                e1 = W[jn + G];
                e2 = W[jn + 2 * G];
                e3 = W[jn + 3 * G];
            }
            term(j, a0, b0);
            term(j + G, a1, b1);
            term(j + 2 * G, a2, b2);
            term(j + 3 * G, a3, b3);
            j = jn;
            if (!more) break;
            a0 = c0; a1 = c1; a2 = c2; a3 = c3;
            b0 = e0; b1 = e1; b2 = e2; b3 = e3;
        }
    }
    for (; j < K; j += G) term(j, D[j], W[j]);
    s[0] = Red::sum(ps);
    s[1] = Red::sum(dps);
    s[2] = Red::sum(ph);
    s[3] = Red::sum(dph);
    if (ZZ) s[4] = Red::sum(zz);
}

// The exclusion window and left/right split of a root's sweeps: the midpoint
// sweep of an interior root excludes both bracketing poles (origin kk), an
// iteration sweep excludes only the origin.
TDE_DEV void sec_split(const SecRoot& r, int kk, int* L1, int* R0) {
    *L1 = r.orgl ? kk : kk + 1;
    *R0 = r.orgl ? kk + 1 : kk + 2;
}

// Z: the merge's z (global); D, W: views of its poles and weights z_j^2
// (global or staged).  The sum of |terms| needed by the stopping test is
// phi - psi (every left term is negative, every right term positive).
template <class Red>
TDE_DEV int secular_root(int k, int K, const double* __restrict__ D, const double* __restrict__ Z,
                         const double* __restrict__ W, double rho, int sub, int G, int cap, int* org_out,
                         double* tau_out) {
    if (K == 1) {
        *org_out = 0;
        *tau_out = rho * Z[0] * Z[0];
        return 0;
    }
    const int kk = (k < K - 1) ? k : K - 2;
    SecRoot r;
    double s[5];
    if (k < K - 1) {
        // Midpoint sweep (origin kk): picks the nearer pole and seeds the first step.
        sec_sweep<Red, false>(K, D, W, D[kk], 0.5 * (D[kk + 1] - D[kk]), kk, kk + 2, sub, G, s);
        if (sec_start_interior(k, D, Z, rho, s[0], s[1], s[2], s[3], &r)) {
            *org_out = r.o;
            *tau_out = r.tau;
            return 0;
        }
    } else {
        double zz = 0.0;
        for (int j = sub; j < K; j += G) zz += W[j];
        zz = Red::sum(zz);
        sec_start_last(K, D, Z, rho, zz, &r);
    }
    for (int it = 1; it <= cap; ++it) {
        int L1, R0;
        sec_split(r, kk, &L1, &R0);
        sec_sweep<Red, false>(K, D, W, D[r.o], r.tau, L1, R0, sub, G, s);
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

// lambda_k - D_i from the compact root (org, tau): (D_org - D_i) + tau.
TDE_DEV double root_minus_pole(const double* __restrict__ D, int org, double tau, int i) {
    return (D[org] - D[i]) + tau;
}

// Loewner recomputation of z_i from the computed roots (appendix, WPROD
// product chains): z_i^2 = prod_k (lambda_k - D_i) / (rho prod_{j!=i}(D_j - D_i)),
// taken as a chain of ratios of like-signed factors near 1:
//   k < i: (lambda_k - D_i)/(D_k - D_i);  i <= k < K-1: (lambda_k - D_i)/(D_{k+1} - D_i);
// times (lambda_{K-1} - D_i).  The sign is that of the input z_i.
template <class Red>
TDE_DEV double lowner_z(int i, int K, const double* __restrict__ D, const double* __restrict__ Z,
                        const int* __restrict__ org, const double* __restrict__ tau, double rho, int sub, int G) {
    const double di = D[i];
    // numerators and denominators multiplied 8 at a time (8 factors of the
    // chain cannot leave the exponent range), one division per chunk
    double prod = 1.0, pn = 1.0, pd = 1.0;
    int c = 0;
    _Pragma("unroll 4") for (int k = sub; k < K; k += G) {
        const double num = (D[org[k]] - di) + tau[k];
        double den;
        if (k < i) den = D[k] - di;
        else if (k < K - 1) den = D[k + 1] - di;
        else den = 1.0;
        pn *= num;
        pd *= den;
        if (++c == 8) {
            prod *= pn / pd;
            pn = 1.0;
            pd = 1.0;
            c = 0;
        }
    }
    prod *= pn / pd;
    prod = Red::prod(prod);
    double z2 = prod / rho;
    double zi = sqrt(fmax(z2, 0.0));
    return (Z[i] < 0.0) ? -zi : zi;
}

// Boundary-row propagation for one root (Section 4.1): parent row entries
// (Q_L (+) Q_R)_sigma y_k with y_k(i) = zhat_i/(D_i - lambda_k), normalised;
// two streamed dot products, no K x K block.
template <class Red>
TDE_DEV void root_rows(int K, const double* __restrict__ D, const double* __restrict__ zh,
                       const double* __restrict__ RL, const double* __restrict__ RH, int org, double tau,
                       int sub, int G, double* bl_out, double* bh_out) {
    const double Do = D[org];
    double ss = 0.0, bl = 0.0, bh = 0.0;
    _Pragma("unroll 4") for (int i = sub; i < K; i += G) {
        const double y = zh[i] * rcp_nr((D[i] - Do) - tau);
        ss = fma(y, y, ss);
        bl = fma(RL[i], y, bl);
        bh = fma(RH[i], y, bh);
    }
    ss = Red::sum(ss);
    bl = Red::sum(bl);
    bh = Red::sum(bh);
    double inv = 1.0 / sqrt(ss);
    *bl_out = bl * inv;
    *bh_out = bh * inv;
}

// ---------------------------------------------------------------------------
// Element-parallel level steps.  Packed position t in [0, N) of a level
// belongs to merge m (mr[m].pk <= t < mr[m].pk + size) at local column
// i = t - mr[m].pk; callers find m (find_merge / find_merge_in).
// ---------------------------------------------------------------------------

// (a3/a4) z~, outer rows and merged sorted order of one child column.
// Left column i: position i + #{right values < x}; right column j:
// j + #{left values <= x} (ties go left first).  Returns the packed position.
// The deflation tolerance of merge R from its children's spectra (the same
// value as merge_tol on the merged poles: the ends of both sorted children).
TDE_DEV double merge_tol_children(const MergeRec& R, const Work& w) {
    const double* lamL = w.lam + R.off;
    const double* lamR = lamL + R.nL;
    const double dmax = fmax(fmax(fabs(lamL[0]), fabs(lamL[R.nL - 1])), fmax(fabs(lamR[0]), fabs(lamR[R.nR - 1])));
    return 8.0 * DBL_EPSILON * fmax(dmax, 1.0);
}

// Writes merged position P: child column c (local index in the parent, left
// child first) with eigenvalue x; z~ and the outer rows from that child's
// boundary rows; (a5) the negligible-z flag, a candidate iff rho~ |z~| > tol.
TDE_DEV int merge_emit(const MergeRec& R, int c, double x, double rho, double sgn, double tol, const Work& w,
                       long long P) {
    const double rs2 = 0.70710678118654752440;  // 1/sqrt(2)
    double z, rl, rh;
    if (c < R.nL) {
        z = w.bhi[R.off + c] * rs2;
        rl = w.blo[R.off + c];
        rh = 0.0;
    } else {
        z = sgn * w.blo[R.off + c] * rs2;
        rl = 0.0;
        rh = w.bhi[R.off + c];
    }
    if (w.xmode) {
        // requested rows: a row reaches this merge from the child that holds it
        const bool cl = c < R.nL;
        const long long mid = R.off + R.nL, end = mid + R.nR;
        rl = (w.xa_row >= R.off && w.xa_row < end && (w.xa_row < mid) == cl) ? w.xa[R.off + c] : 0.0;
        rh = (w.xb_row >= R.off && w.xb_row < end && (w.xb_row < mid) == cl) ? w.xb[R.off + c] : 0.0;
    }
    w.D[P] = x;
    w.Z[P] = z;
    w.RL[P] = rl;
    w.RH[P] = rh;
    w.src[P] = c;
    const int flag = (rho * fabs(z) > tol) ? 1 : 0;
    w.st[P] = flag;
    return flag;
}

// Partition point of an ascending array (how many values are < x, or <= x):
// a binary search, or with Wide an 8-way search first, 7 probes read at once
// (independent loads) each round, so a list of n values costs about log8(n)
// dependent reads instead of log2(n) -- the better choice where few threads
// run and each waits on its chain of reads, the worse where many threads
// share the memory system.  Both give the same index.
template <bool LE, bool Wide, class Val>
TDE_DEV int count_part(const Val& v, int n, double x) {
    int lo = 0, hi = n;
    while (Wide && hi - lo > 8) {
        const long long r = hi - lo;
        double pv[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) pv[k] = v(lo + (int)((r * (k + 1)) >> 3));
        int c = 0;
#pragma unroll
        for (int k = 0; k < 7; ++k) c += (LE ? (pv[k] <= x) : (pv[k] < x)) ? 1 : 0;
        // the answer lies after the c-th probe and at or before the (c+1)-th
        const int nlo = c ? lo + (int)((r * c) >> 3) + 1 : lo;
        const int nhi = (c < 7) ? lo + (int)((r * (c + 1)) >> 3) : hi;
        lo = nlo;
        hi = nhi;
    }
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double vm = v(mid);
        if (LE ? (vm <= x) : (vm < x)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
template <bool Wide = false>
TDE_DEV int count_lt(const double* __restrict__ v, int n, double x) {
    return count_part<false, Wide>([v](int i) { return v[i]; }, n, x);
}
template <bool Wide = false>
TDE_DEV int count_le(const double* __restrict__ v, int n, double x) {
    return count_part<true, Wide>([v](int i) { return v[i]; }, n, x);
}

TDE_DEV long long body_merge(long long t, int m, const MergeRec* __restrict__ mr,
                             const double* __restrict__ e, const unsigned long long* __restrict__ pmax,
                             const Work& w, int* flag_out) {
    const MergeRec R = mr[m];
    const int i = (int)(t - R.pk);
    double sgn;
    const double rho = merge_rho(R, e, pmax, &sgn);
    const double* lamL = w.lam + R.off;
    const double* lamR = lamL + R.nL;
    const double tol = merge_tol_children(R, w);
    int pos;
    double x;
    if (i < R.nL) {
        x = lamL[i];
        pos = i + count_lt(lamR, R.nR, x);
    } else {
        const int j = i - R.nL;
        x = lamR[j];
        pos = j + count_le(lamL, R.nL, x);
    }
    const long long P = R.pk + pos;
    *flag_out = merge_emit(R, i, x, rho, sgn, tol, w, P);
    return P;
}



// One step of a run: the running column *cur (left) against the next
// candidate nx.  If the pair passes the close test on the current values it
// is rotated by the Givens rotation that zeroes cur's z (c = z_nx/t,
// s = z_cur/t, t = hypot): *def receives the deflated column (pole
// c^2 D_cur + s^2 D_nx, z = 0, rows c r_cur - s r_nx) and *cur becomes the
// survivor (pole s^2 D_cur + c^2 D_nx, z = t, rows s r_cur + c r_nx); returns
// true.  Otherwise returns false and leaves *cur unchanged.  Both new poles
// are convex combinations of D_cur <= D_nx and are clamped into that interval
// so rounding cannot break the ascending order the assembly merges on.
TDE_DEV bool run_step(RunState* cur, const RunState& nx, double tol, RunState* def, double* cc, double* ss) {
#pragma clang fp contract(off)
    const double tt = hypot(cur->Z, nx.Z);
    const double c = nx.Z / tt, sn = cur->Z / tt;
    *cc = c;
    *ss = sn;
    if (!(fabs((nx.D - cur->D) * c * sn) <= tol)) return false;
    def->D = fmin(fmax(c * c * cur->D + sn * sn * nx.D, cur->D), nx.D);
    def->Z = 0.0;
    def->L = c * cur->L - sn * nx.L;
    def->H = c * cur->H - sn * nx.H;
    RunState sv;
    sv.D = fmin(fmax(sn * sn * cur->D + c * c * nx.D, cur->D), nx.D);
    sv.Z = tt;
    sv.L = sn * cur->L + c * nx.L;
    sv.H = sn * cur->H + c * nx.H;
    *cur = sv;
    return true;
}

// (a5) close poles.  Candidate g (the g-th non-negligible column of the level)
// starts a run if it passes the close test with its successor but not with
// its predecessor, both tested on the unrotated values; the run extends while
// consecutive candidates keep passing.  The run's owner walks the run left to
// right, re-testing each pair on the current (rotated) values, and deflates
// the left column of every rotated pair.  All tests read the unrotated arrays
// (D, Z, RL, RH) and every candidate's final values go to (D2, Z2, RL2, RH2),
// so runs proceed in parallel without races; a candidate outside every run is
// copied through by its own thread.  on_rotate(p) is called for each column
// rotated away.
TDE_DEV bool cand_close(const Work& w, long long a, long long b, double tol) {
    const long long pa = w.nnpos[a], pb = w.nnpos[b];
    return close_pair(w.D[pa], w.Z[pa], w.D[pb], w.Z[pb], tol);
}

template <class OnRotate>
TDE_DEV void body_runs(long long g, int m, const MergeRec* __restrict__ mr, const Work& w, OnRotate on_rotate) {
    const int* __restrict__ nnpos = w.nnpos;
    const long long t = nnpos[g];
    const MergeRec R = mr[m];
    const int s = R.nL + R.nR;
    const long long gs = w.scanC[R.pk], ge = w.scanC[R.pk + s];
    const double tol = merge_tol(w.D, R.pk, s);
    const bool cl_next = (g + 1 < ge) && cand_close(w, g, g + 1, tol);
    const bool cl_prev = (g > gs) && cand_close(w, g - 1, g, tol);
    if (cl_prev) return;  // inside a run owned by an earlier candidate
    if (!cl_next) {       // not in any run: copy through
        w.D2[t] = w.D[t];
        w.Z2[t] = w.Z[t];
        w.RL2[t] = w.RL[t];
        w.RH2[t] = w.RH[t];
        return;
    }
    long long r = g + 1;
    while (r + 1 < ge && cand_close(w, r, r + 1, tol)) ++r;
    long long pc = t;
    RunState cur{w.D[pc], w.Z[pc], w.RL[pc], w.RH[pc]};
    for (long long j = g + 1; j <= r; ++j) {
        const long long pj = nnpos[j];
        const RunState nx{w.D[pj], w.Z[pj], w.RL[pj], w.RH[pj]};
        RunState def;
        double c, sn;
        if (run_step(&cur, nx, tol, &def, &c, &sn)) {
            w.D2[pc] = def.D;
            w.Z2[pc] = 0.0;
            w.RL2[pc] = def.L;
            w.RH2[pc] = def.H;
            w.st[pc] = 2;
            on_rotate(pc);
        } else {
            w.D2[pc] = cur.D;
            w.Z2[pc] = cur.Z;
            w.RL2[pc] = cur.L;
            w.RH2[pc] = cur.H;
            cur = nx;
        }
        pc = pj;
    }
    w.D2[pc] = cur.D;
    w.Z2[pc] = cur.Z;
    w.RL2[pc] = cur.L;
    w.RH2[pc] = cur.H;
    // The rotated-away columns of a run join their own list, ascending in
    // position order: sort them among the run's rotated positions (only
    // columns g..r-1 can be rotated away).  Their values lie in [D_g, D_r],
    // so the lists of different runs stay ordered.
    for (long long j = g; j < r; ++j) {
        const long long pj = nnpos[j];
        if (w.st[pj] != 2) continue;
        const double kD = w.D2[pj], kL = w.RL2[pj], kH = w.RH2[pj];
        long long h = j;
        for (long long q = j - 1; q >= g; --q) {
            const long long pq = nnpos[q];
            if (w.st[pq] != 2) continue;
            if (w.D2[pq] <= kD) break;
            const long long ph = nnpos[h];
            w.D2[ph] = w.D2[pq]; w.RL2[ph] = w.RL2[pq]; w.RH2[ph] = w.RH2[pq];
            h = q;
        }
        const long long ph = nnpos[h];
        w.D2[ph] = kD; w.RL2[ph] = kL; w.RH2[ph] = kH;
    }
}

// Largest m with scan[mr[m].pk] <= g: the merge owning active column g.
TDE_DEV int find_merge_active(const MergeRec* __restrict__ mr, int M, const int* __restrict__ scan, long long g) {
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (scan[mr[mid].pk] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Root-parallel steps.  m is the merge owning active column g (recorded at
// compaction).  The merge's active arrays are read through views: element
// ks + j of the level-wide array is view[ks + j - voff], so a caller can pass
// either the level-wide arrays (voff = 0) or a copy of a window of them staged
// in LDS (voff = first staged index).
struct MergeSpan {
    long long ks;  // first active column of the merge
    int K;         // active columns
};
TDE_DEV MergeSpan merge_span(const MergeRec& R, const int* __restrict__ scan) {
    MergeSpan sp;
    sp.ks = scan[R.pk];
    sp.K = (int)(scan[R.pk + R.nL + R.nR] - sp.ks);
    return sp;
}

// (a6) one secular root (lane sub of a G-lane group).
template <class Red>
TDE_DEV int body_secular(long long g, int m, const MergeRec* __restrict__ mr, const double* __restrict__ e,
                         const unsigned long long* __restrict__ pmax, const Work& w, int sub, int G,
                         const double* __restrict__ Dv, const double* __restrict__ Wv, long long voff) {
    const MergeRec R = mr[m];
    const MergeSpan sp = merge_span(R, w.scan);
    double sgn;
    const double rho = merge_rho(R, e, pmax, &sgn);
    int o;
    double tau;
    const long long b = sp.ks - voff;
    const int it =
        secular_root<Red>((int)(g - sp.ks), sp.K, Dv + b, w.Za + sp.ks, Wv + b, rho, sub, G, w.sec_cap, &o, &tau);
    if (sub == 0) {
        w.org[g] = o;
        w.tau[g] = tau;
        w.rootval[g] = Dv[b + o] + tau;
    }
    return it;
}

// (a7) Loewner z-hat for active pole g (non-root merges only).
template <class Red>
TDE_DEV void body_lowner(long long g, int m, const MergeRec* __restrict__ mr, const double* __restrict__ e,
                         const unsigned long long* __restrict__ pmax, const Work& w, int sub, int G,
                         const double* __restrict__ Dv, const int* __restrict__ orgv,
                         const double* __restrict__ tauv, long long voff, bool with_root = false) {
    const MergeRec R = mr[m];
    if ((R.flags & MF_ROOT) && !with_root && !w.rows_out) return;
    const MergeSpan sp = merge_span(R, w.scan);
    double sgn;
    const double rho = merge_rho(R, e, pmax, &sgn);
    const long long b = sp.ks - voff;
    const double zh = lowner_z<Red>((int)(g - sp.ks), sp.K, Dv + b, w.Za + sp.ks, orgv + b, tauv + b, rho, sub, G);
    if (sub == 0) w.zhat[g] = zh;
}

// (a7) parent boundary-row entries of active root g (non-root merges only).
template <class Red>
TDE_DEV void body_rows(long long g, int m, const MergeRec* __restrict__ mr, const Work& w, int sub, int G,
                       const double* __restrict__ Dv, const double* __restrict__ zhv,
                       const double* __restrict__ RLv, const double* __restrict__ RHv, long long voff) {
    const MergeRec R = mr[m];
    if ((R.flags & MF_ROOT) && !w.rows_out) return;
    const MergeSpan sp = merge_span(R, w.scan);
    const long long b = sp.ks - voff;
    double bl, bh;
    root_rows<Red>(sp.K, Dv + b, zhv + b, RLv + b, RHv + b, w.org[g], w.tau[g], sub, G, &bl, &bh);
    if (sub == 0) {
        w.PBL[g] = bl;
        w.PBH[g] = bh;
    }
}

// (a9) parent assembly: merge three ascending lists -- the roots, the
// negligible-z columns and the rotated-away columns -- into the parent's
// spectrum, in place (or the scaled-back eigenvalues for a top merge).  Ties
// order roots before rotated before negligible columns.
//
// Roots given as (origin index, tau) pairs, ascending: how many are <= x.
template <bool Wide>
TDE_DEV int roots_cmp_count(const double* __restrict__ Da, const int* __restrict__ og,
                            const double* __restrict__ ta, int K, double x) {
    return count_part<true, Wide>([Da, og, ta](int i) { return Da[og[i]] + ta[i]; }, K, x);
}

// Rows mode: first and last entries of the unit eigenvector of an output
// eigenvalue, signed so that the first entry is >= 0 (the last when the first
// is 0).
TDE_DEV void store_rows(const Work& w, long long P, double bl, double bh) {
    const double sg = (!w.rows_raw && (bl < 0.0 || (bl == 0.0 && bh < 0.0))) ? -1.0 : 1.0;
    if (w.qfirst) w.qfirst[P] = sg * bl;
    if (w.qlast) w.qlast[P] = sg * bh;
}

//
// part 1 places only the roots (i < K), part 2 only the deflated columns, so
// that the roots can be placed by the kernels that finish them.
template <bool Wide = false>
TDE_DEV void body_assemble(long long t, int m, const MergeRec* __restrict__ mr,
                           const unsigned long long* __restrict__ pmax, const Work& w, double* __restrict__ out,
                           int part = 0) {
    const MergeRec R = mr[m];
    const int s = R.nL + R.nR;
    const int i = (int)(t - R.pk);
    const long long ks = w.scan[R.pk];
    const int K = (int)(w.scan[R.pk + s] - ks);
    if ((part == 1 && i >= K) || (part == 2 && i < K)) return;
    const long long rs = w.scanR[R.pk];
    const int nr = (int)(w.scanR[R.pk + s] - rs);
    const long long ns = R.pk - ks - rs;
    const int nn = s - K - nr;
    const double* rv = w.rootval + ks;  // D_org + tau of each root, ascending
    const double* Dr = w.Dr + rs;
    const double* Dd = w.Dd + ns;
    const bool root = (R.flags & MF_ROOT) != 0;
    const bool rows = !root || w.rows_out;
    int pos;
    double val, bl = 0.0, bh = 0.0;
    if (i < K) {
        val = rv[i];
        pos = i + count_lt<Wide>(Dr, nr, val) + count_lt<Wide>(Dd, nn, val);
        if (rows) { bl = w.PBL[ks + i]; bh = w.PBH[ks + i]; }
    } else if (i < K + nr) {
        const int q = i - K;
        val = Dr[q];
        pos = q + count_le<Wide>(rv, K, val) + count_lt<Wide>(Dd, nn, val);
        if (rows) { bl = w.RLr[rs + q]; bh = w.RHr[rs + q]; }
    } else {
        const int q = i - K - nr;
        val = Dd[q];
        pos = q + count_le<Wide>(rv, K, val) + count_le<Wide>(Dr, nr, val);
        if (rows) { bl = w.RLd[ns + q]; bh = w.RHd[ns + q]; }
    }
    const long long P = R.off + pos;
    if (w.xmode) {
        const bool ha = w.xa_row >= R.off && w.xa_row < R.off + s;
        const bool hb = w.xb_row >= R.off && w.xb_row < R.off + s;
        if (root) {
            if (ha && w.xq_a) w.xq_a[P] = bl;
            if (hb && w.xq_b) w.xq_b[P] = bh;
        } else {
            if (ha) w.xa[P] = bl;
            if (hb) w.xb[P] = bh;
        }
        return;
    }
    if (root) {
        out[P] = val * scale_of(pmax[R.prob]);
        if (w.rows_out) store_rows(w, P, bl, bh);
    } else {
        w.lam[P] = val;
        w.blo[P] = bl;
        w.bhi[P] = bh;
    }
}

// Leaf load + tear + solve for one lane.  The tear subtracts |beta| from the
// two diagonal entries adjacent to every torn coupling (Eq. dc-split with
// u = e_m + sign(beta) e_{m+1}, rho = |beta|).
TDE_DEV int body_leaf(const LeafRec& L, const double* __restrict__ d, const double* __restrict__ e,
                      const unsigned long long* __restrict__ pmax, const Work& w, double* __restrict__ out,
                      double* sd, double* se, double* s0, double* s1, int st, unsigned* nrot) {
    const double inv = 1.0 / scale_of(pmax[L.prob]);
    const int nl = L.size;
    for (int i = 0; i < nl; ++i) {
        double di = d[L.off + i] * inv;
        if (i == 0 && (L.flags & LF_TEAR_LEFT)) di -= fabs(e[L.off - 1] * inv);
        if (i == nl - 1 && (L.flags & LF_TEAR_RIGHT)) di -= fabs(e[L.off + nl - 1] * inv);
        sd[i * st] = di;
        se[i * st] = (i + 1 < nl) ? e[L.off + i] * inv : 0.0;
    }
    // tracked rows: 0 and l-1, or in a requested-rows pass the requested rows
    // the leaf holds
    const bool ha = w.xmode && w.xa_row >= L.off && w.xa_row < L.off + nl;
    const bool hb = w.xmode && w.xb_row >= L.off && w.xb_row < L.off + nl;
    int status = leaf_ql(nl, sd, se, s0, s1, st, nrot, ha ? (int)(w.xa_row - L.off) : 0,
                         hb ? (int)(w.xb_row - L.off) : nl - 1);
    if (w.xmode) {
        double* da = (L.flags & LF_WHOLE) ? w.xq_a : w.xa;
        double* db = (L.flags & LF_WHOLE) ? w.xq_b : w.xb;
        for (int i = 0; i < nl; ++i) {
            if (ha && da) da[L.off + i] = s0[i * st];
            if (hb && db) db[L.off + i] = s1[i * st];
        }
        return status;
    }
    if (L.flags & LF_WHOLE) {
        const double sc = 1.0 / inv;
        for (int i = 0; i < nl; ++i) {
            out[L.off + i] = sd[i * st] * sc;
            if (w.rows_out) store_rows(w, L.off + i, s0[i * st], s1[i * st]);
        }
    } else {
        for (int i = 0; i < nl; ++i) {
            w.lam[L.off + i] = sd[i * st];
            w.blo[L.off + i] = s0[i * st];
            w.bhi[L.off + i] = s1[i * st];
        }
    }
    return status;
}

}  // namespace tde
