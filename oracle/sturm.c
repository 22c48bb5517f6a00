/*
 * ORACLE -- test infrastructure only.  Nothing on the product path may link,
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.
 *
 * What it computes: all (or selected) eigenvalues of a real symmetric
 * tridiagonal matrix T (diagonal d[0..n), off-diagonal e[0..n-1)), ascending,
 * in IEEE binary64.  The paper's theorem on boundary-row D&C (Section 3.2,
 * "BR computes the same eigenvalues as conventional D&C") says the method
 * returns the spectrum of T; the plainest independent definition of that
 * spectrum used here is Sturm-sequence bisection (Section 2.1 lists bisection
 * among the standard tridiagonal solvers):
 *
 *   count(x) = #{ eigenvalues of T that are < x }
 *            = number of negative pivots q_i of the LDL^T factorisation of
 *              T - xI:   q_0 = d_0 - x,  q_i = (d_i - x) - e_{i-1}^2 / q_{i-1}.
 *
 *   The k-th smallest eigenvalue (k = 0..n-1) is the point where count
 *   steps from <= k to > k; bisection on a Gershgorin interval finds it.
 *
 * Conventions (not fixed by the paper; restated in the design doc):
 *  - Input is first scaled by an exact power of two so that its largest entry
 *    lies in (1/2, 1]; eigenvalues are scaled back at the end (exact).
 *  - A pivot smaller in magnitude than pivmin = DBL_MIN * max(1, max e_i^2) is
 *    replaced by -pivmin (so a zero pivot counts as negative, i.e. x is taken
 *    as lying just above an eigenvalue it hits exactly).
 *  - Bisection stops when the interval can no longer be split, when its width
 *    is <= 2 eps max(|a|,|b|), or when it is <= eps*||T||/1024 (an absolute
 *    floor far below the accuracy the Sturm count itself can certify).
 *  - Non-finite input returns -1 and writes nothing.
 *
 * Plain loops, OpenMP only across independent eigenvalue indices.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int all_finite(int64_t n, const double* d, const double* e) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(d[i])) return 0;
    for (int64_t i = 0; i + 1 < n; ++i)
        if (!isfinite(e[i])) return 0;
    return 1;
}

/* 2^ceil(log2(max |entry|)); 1 for the zero matrix. */
static double pow2_scale(int64_t n, const double* d, const double* e) {
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) mx = fmax(mx, fabs(d[i]));
    for (int64_t i = 0; i + 1 < n; ++i) mx = fmax(mx, fabs(e[i]));
    if (mx == 0.0) return 1.0;
    int ex;
    double fr = frexp(mx, &ex); /* mx = fr * 2^ex, fr in [1/2, 1) */
    (void)fr;
    return ldexp(1.0, ex);      /* mx / scale in [1/2, 1) */
}

typedef struct {
    int64_t n;
    double* d;    /* scaled diagonal */
    double* e2;   /* squared scaled off-diagonal, length n-1 */
    double pivmin;
    double glo, ghi; /* Gershgorin interval, widened */
    double tnorm;    /* ||T||_1 of the scaled matrix */
    double scale;
} scaled_t;

static int64_t sturm_count_scaled(const scaled_t* s, double x) {
    int64_t cnt = 0;
    double q = s->d[0] - x;
    if (fabs(q) < s->pivmin) q = -s->pivmin;
    if (q < 0.0) ++cnt;
    for (int64_t i = 1; i < s->n; ++i) {
        q = (s->d[i] - x) - s->e2[i - 1] / q;
        if (fabs(q) < s->pivmin) q = -s->pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

/* The same count at CW points at once: each point runs exactly the scalar
 * recurrence above (same operations in the same order), the points only
 * share the loop so that their independent divisions overlap. */
#define CW 8
static void sturm_count_scaled_group(const scaled_t* s, const double* x, int64_t* cnt) {
    double q[CW];
    int64_t c[CW];
    for (int j = 0; j < CW; ++j) {
        q[j] = s->d[0] - x[j];
        if (fabs(q[j]) < s->pivmin) q[j] = -s->pivmin;
        c[j] = (q[j] < 0.0) ? 1 : 0;
    }
    for (int64_t i = 1; i < s->n; ++i) {
        const double di = s->d[i], e2 = s->e2[i - 1];
        for (int j = 0; j < CW; ++j) {
            double t = (di - x[j]) - e2 / q[j];
            if (fabs(t) < s->pivmin) t = -s->pivmin;
            c[j] += (t < 0.0) ? 1 : 0;
            q[j] = t;
        }
    }
    for (int j = 0; j < CW; ++j) cnt[j] = c[j];
}

static int setup(scaled_t* s, int64_t n, const double* d, const double* e) {
    s->n = n;
    s->scale = pow2_scale(n, d, e);
    s->d = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    s->e2 = (double*)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    if (!s->d || !s->e2) return -2;
    double inv = 1.0 / s->scale;
    double maxe2 = 0.0;
    for (int64_t i = 0; i < n; ++i) s->d[i] = d[i] * inv;
    for (int64_t i = 0; i + 1 < n; ++i) {
        double t = e[i] * inv;
        s->e2[i] = t * t;
        if (s->e2[i] > maxe2) maxe2 = s->e2[i];
    }
    s->pivmin = DBL_MIN * fmax(1.0, maxe2);
    /* Gershgorin: every eigenvalue lies in some [d_i - r_i, d_i + r_i]. */
    double glo = INFINITY, ghi = -INFINITY, tn = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        if (i > 0) r += fabs(e[i - 1] * inv);
        if (i + 1 < n) r += fabs(e[i] * inv);
        glo = fmin(glo, s->d[i] - r);
        ghi = fmax(ghi, s->d[i] + r);
        tn = fmax(tn, fabs(s->d[i]) + r);
    }
    double w = 2.0 * DBL_EPSILON * fmax(fabs(glo), fabs(ghi)) + 2.0 * s->pivmin;
    s->glo = glo - w;
    s->ghi = ghi + w;
    s->tnorm = tn;
    return 0;
}

static void teardown(scaled_t* s) {
    free(s->d);
    free(s->e2);
}

/* k-th smallest eigenvalue (0-based) of the scaled matrix, by bisection. */
static double kth_scaled(const scaled_t* s, int64_t k) {
    if (s->tnorm == 0.0) return 0.0; /* T = 0: every eigenvalue is 0 */
    double a = s->glo, b = s->ghi;
    double floor_abs = DBL_EPSILON * s->tnorm / 1024.0;
    for (int it = 0; it < 4000; ++it) {
        double width = b - a;
        if (width <= 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) || width <= floor_abs) break;
        double m = a + 0.5 * width;
        if (m <= a || m >= b) break;
        if (sturm_count_scaled(s, m) <= k)
            a = m; /* at most k eigenvalues below m: lambda_k >= m */
        else
            b = m; /* more than k below m: lambda_k < m */
    }
    return a + 0.5 * (b - a);
}

/* All eigenvalues, ascending.  Returns 0, -1 (non-finite input), -2 (no memory). */
int oracle_eigvals(int64_t n, const double* d, const double* e, double* lam) {
    if (n < 0) return -3;
    if (n == 0) return 0;
    if (!all_finite(n, d, e)) return -1;
    scaled_t s;
    if (setup(&s, n, d, e)) { teardown(&s); return -2; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) lam[k] = kth_scaled(&s, k) * s.scale;
    teardown(&s);
    return 0;
}

/* Selected eigenvalues lam[j] = lambda_{ks[j]} (0-based, ascending order of the spectrum). */
int oracle_eigvals_index(int64_t n, const double* d, const double* e, int64_t nk, const int64_t* ks,
                         double* lam) {
    if (n < 0 || nk < 0) return -3;
    if (n == 0 || nk == 0) return 0;
    if (!all_finite(n, d, e)) return -1;
    for (int64_t j = 0; j < nk; ++j)
        if (ks[j] < 0 || ks[j] >= n) return -3;
    scaled_t s;
    if (setup(&s, n, d, e)) { teardown(&s); return -2; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < nk; ++j) lam[j] = kth_scaled(&s, ks[j]) * s.scale;
    teardown(&s);
    return 0;
}

/* Sturm counts at arbitrary points: cnt[j] = #{eigenvalues < x[j]} (with the
 * pivmin convention above).  Used to certify a computed spectrum at sizes
 * where bisecting every eigenvalue is too slow: if for every k
 * count(mu_k - t) <= k < count(mu_k + t) then |mu_k - lambda_k| <= t. */
int oracle_counts(int64_t n, const double* d, const double* e, int64_t np, const double* x,
                  int64_t* cnt) {
    if (n < 0 || np < 0) return -3;
    if (np == 0) return 0;
    if (n == 0) {
        for (int64_t j = 0; j < np; ++j) cnt[j] = 0;
        return 0;
    }
    if (!all_finite(n, d, e)) return -1;
    scaled_t s;
    if (setup(&s, n, d, e)) { teardown(&s); return -2; }
    const int64_t ng = np / CW;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t gi = 0; gi < ng; ++gi) {
        double xs[CW];
        for (int j = 0; j < CW; ++j) xs[j] = x[gi * CW + j] / s.scale;
        sturm_count_scaled_group(&s, xs, cnt + gi * CW);
    }
    for (int64_t j = ng * CW; j < np; ++j) cnt[j] = sturm_count_scaled(&s, x[j] / s.scale);
    teardown(&s);
    return 0;
}

/* As oracle_counts, one point at a time (the scalar recurrence only); kept to
 * check that the grouped form above returns the same counts. */
int oracle_counts_scalar(int64_t n, const double* d, const double* e, int64_t np, const double* x,
                         int64_t* cnt) {
    if (n < 0 || np < 0) return -3;
    if (np == 0) return 0;
    if (n == 0) {
        for (int64_t j = 0; j < np; ++j) cnt[j] = 0;
        return 0;
    }
    if (!all_finite(n, d, e)) return -1;
    scaled_t s;
    if (setup(&s, n, d, e)) { teardown(&s); return -2; }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < np; ++j) cnt[j] = sturm_count_scaled(&s, x[j] / s.scale);
    teardown(&s);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
