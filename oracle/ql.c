/*
 * CPU BASELINE -- test/benchmark infrastructure only (never on the product path).
 *
 * Plain eigenvalue-only implicit QL with a Wilkinson shift for a real
 * symmetric tridiagonal matrix: the sequential QR/QL family the paper compares
 * boundary-row D&C against (Section 2.1 and the QR/QL baseline of Section 5.2).
 *
 * Written from the mathematics of the implicit symmetric QR step with a
 * Wilkinson shift as Golub and Van Loan state it (Matrix Computations, 4th ed.,
 * Section 8.3, Algorithm 8.3.2), mirrored into its QL form: the shift comes
 * from the top 2x2 block of the active block, the first plane rotation from
 * the shifted last column, and the bulge it creates is chased upward; the top
 * coupling converges and the block shrinks from the top.
 *
 * Rotation in plane (k, k+1) with cosine c and sine s: rows k and k+1 become
 * c r_k - s r_(k+1) and s r_k + c r_(k+1); applied from both sides,
 *   d_k'     = c^2 d_k - 2 c s e_k + s^2 d_(k+1)
 *   d_(k+1)' = s^2 d_k + 2 c s e_k + c^2 d_(k+1)
 *   e_k'     = c s (d_k - d_(k+1)) + (c^2 - s^2) e_k
 *   e_(k-1)' = c e_(k-1), and a bulge s e_(k-1) appears at (k-1, k+1).
 * With c^2 + s^2 = 1 the first three are evaluated in difference form,
 * w = s (d_k - d_(k+1)) + 2 c e_k: d_k' = d_k - s w, d_(k+1)' = d_(k+1) + s w,
 * e_k' = c w - e_k (the trace is kept exactly, no c^2 / s^2 cancellation).
 * The rotation of the chase that removes a bulge b at (k, k+2) has
 * c = e_(k+1)/r, s = b/r, r = hypot(b, e_(k+1)), and leaves e_(k+1)' = r.
 *
 * Output eigenvalues are sorted ascending.  Returns 0, -1 on non-finite input,
 * -2 when out of memory, 1 if some eigenvalue did not converge in 60 steps.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Eigenvalue of [a f; f g] nearer to a (Wilkinson shift), overflow-safe. */
static double wilkinson_shift(double a, double f, double g) {
    if (f == 0.0) return a;
    double h = (g - a) / (2.0 * f);
    double r = hypot(h, 1.0);
    return a - f / (h + (h >= 0.0 ? r : -r));
}

/* One implicit QL step with shift mu on the unreduced block [l, m]. */
static void ql_step(double* d, double* e, int64_t l, int64_t m, double mu) {
    double c, s, r;
    /* first rotation: annihilates the (m-1, m) entry of T - mu I */
    {
        double x = d[m] - mu, y = e[m - 1];
        r = hypot(x, y);
        c = (r == 0.0) ? 1.0 : x / r;
        s = (r == 0.0) ? 0.0 : y / r;
    }
    double bulge = 0.0;
    for (int64_t k = m - 1; k >= l; --k) {
        if (k < m - 1) {
            /* rotation that removes the bulge at (k, k+2) */
            r = hypot(bulge, e[k + 1]);
            c = (r == 0.0) ? 1.0 : e[k + 1] / r;
            s = (r == 0.0) ? 0.0 : bulge / r;
            e[k + 1] = r;
        }
        /* the 2x2 update in difference form (trace kept exactly):
         * w = s (a - g) + 2 c f, d_k' = a - s w, d_(k+1)' = g + s w, e_k' = c w - f */
        double a = d[k], g = d[k + 1], f = e[k];
        double w = s * (a - g) + 2.0 * c * f;
        d[k] = a - s * w;
        d[k + 1] = g + s * w;
        e[k] = c * w - f;
        if (k > l) {
            bulge = s * e[k - 1];
            e[k - 1] = c * e[k - 1];
        }
    }
}

int ql_eigvals(int64_t n, const double* d_in, const double* e_in, double* lam) {
    if (n <= 0) return 0;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(d_in[i])) return -1;
    for (int64_t i = 0; i + 1 < n; ++i)
        if (!isfinite(e_in[i])) return -1;
    double* d = lam;
    double* e = (double*)calloc((size_t)n, sizeof(double)); /* e[i] couples i, i+1; e[n-1] = 0 */
    if (!e) return -2;
    memcpy(d, d_in, sizeof(double) * (size_t)n);
    for (int64_t i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    int status = 0;
    for (int64_t l = 0; l < n; ++l) {
        int steps = 0;
        for (;;) {
            /* end m of the unreduced block starting at l: first negligible coupling */
            int64_t m = l;
            while (m + 1 < n && fabs(e[m]) > DBL_EPSILON * (fabs(d[m]) + fabs(d[m + 1]))) ++m;
            if (m + 1 < n) e[m] = 0.0;
            if (m == l) break; /* d[l] has converged */
            if (++steps > 60) {
                status = 1;
                break;
            }
            ql_step(d, e, l, m, wilkinson_shift(d[l], e[l], d[l + 1]));
        }
    }
    free(e);
    qsort(lam, (size_t)n, sizeof(double), cmp_double);
    return status;
}
