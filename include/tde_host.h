/*
 * tde_host -- boundary-row divide and conquer for the eigenvalues of a real
 * symmetric tridiagonal matrix on the host CPU (OpenMP), FP64.
 *
 * The paper's CPU design (Zhan & Zhang, Section 4.2) as a second host
 * baseline beside the GPU library: a driver that validates the input, splits
 * at negligible couplings, scales every unreduced block by a power of two and
 * solves small blocks by implicit QR; larger blocks go to BR D&C (Algorithm 1)
 * with the first and last eigenvector rows of every node (BLO/BHI) as the only
 * vector state, leaves solved by implicit QR tracking those two rows, and the
 * merges of one tree level run in parallel with disjoint workspace slices.
 * It is a separate library (libtde_host.so, built with g++ -fopenmp) and is
 * never called by the GPU entry points of tde.h.
 *
 * All pointers are HOST pointers; the caller owns every buffer.  Synchronous;
 * nothing is printed; no exceptions cross this interface.
 */
#ifndef TDE_HOST_H
#define TDE_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDE_HOST_OK 0
#define TDE_HOST_EINVAL (-1)     /* bad size, pointer, workspace or thread count */
#define TDE_HOST_ENONFINITE (-4) /* NaN or Inf in d or e */
#define TDE_HOST_ENOCONV 1       /* a QR or secular iteration hit its cap (results still written) */

/* Workspace of tde_host_eigvals for order n: *lwork doubles and *liwork ints
 * (16 n and 2 n: linear in n, nothing per thread).  TDE_HOST_OK or EINVAL. */
int tde_host_workspace(int64_t n, int64_t* lwork, int64_t* liwork);

/* All eigenvalues of T (diagonal d[n], off-diagonal e[n-1], e[i] coupling rows
 * i and i+1), ascending, into lambda[n].
 *   work[lwork], iwork[liwork]  workspace of at least tde_host_workspace's sizes
 *   nthreads                    OpenMP threads (0 = the OpenMP default)
 * Returns TDE_HOST_OK, a negative code for bad arguments / non-finite input
 * (nothing written), or TDE_HOST_ENOCONV. */
int tde_host_eigvals(const double* d, const double* e, int64_t n, double* lambda, double* work, int64_t lwork,
                     int* iwork, int64_t liwork, int nthreads);

#ifdef __cplusplus
}
#endif

#endif /* TDE_HOST_H */
