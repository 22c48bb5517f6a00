/*
 * CPU BASELINE -- test/benchmark infrastructure only (never on the product path).
 *
 * Plain eigenvalue-only implicit QL with a Wilkinson-type shift for a real
 * symmetric tridiagonal matrix: the sequential QR/QL family the paper compares
 * boundary-row D&C against (Section 2.1 and the QR/QL baseline of Section 5.2).
 * This is the textbook implicit-shift QL iteration (Bowdler, Martin, Reinsch
 * and Wilkinson, 1968), written out plainly; no square-root-free tricks.
 *
 *   For the active block [l, m]: pick the shift from the leading 2x2 block,
 *   chase the bulge upward with plane rotations from row m-1 to row l,
 *   and shrink the block once e[l] is negligible.
 *
 * Output eigenvalues are sorted ascending.  Returns 0, -1 on non-finite input,
 * 1 if some eigenvalue did not converge in 60 sweeps.
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
        int iter = 0;
        for (;;) {
            /* Smallest m >= l with a negligible coupling e[m] (or m = n-1). */
            int64_t m = l;
            for (; m + 1 < n; ++m) {
                double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= DBL_EPSILON * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) { status = 1; break; }
            /* Shift: eigenvalue of the leading 2x2 block [d_l e_l; e_l d_{l+1}] nearer d_l. */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int64_t i;
            for (i = m - 1; i >= l; --i) {
                double f = s * e[i];
                double b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) { /* exact deflation inside the sweep */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    free(e);
    qsort(lam, (size_t)n, sizeof(double), cmp_double);
    return status;
}
