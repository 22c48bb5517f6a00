// Dense front end: blocked Householder reduction of a symmetric matrix to
// tridiagonal form (Section 2.1), feeding the boundary-row solver.
#pragma once
#include <stddef.h>

namespace tde {

constexpr int kNb = 32;  // panel width (reflectors per trailing update)

// Scratch of one reduction of an n x n matrix: the panel's reflectors V and
// the matching W (n x kNb each, column-major, global row index), the product
// y = A22 v, the panel's tau, the column's dot products W^T v and V^T v, the
// next reflector unscaled (ua) with its scale and the last w's alpha (sc),
// the row-parallel kernels' per-workgroup partial sums and their two arrival
// tickets, and the tridiagonal's d[n], e[n].
struct DenseWork {
    double* V;
    double* W;
    double* y;
    double* tau;
    double* sdot;
    double* ua;
    double* sc;
    double* part;
    unsigned* ticket;
    double* d;
    double* e;
};

// Layout of DenseWork at base (size only when base == nullptr).
size_t dense_layout(long long n, char* base, DenseWork* dw);

// Enqueue the reduction of A (n x n, column-major, leading dimension lda,
// both triangles, overwritten) to d, e of dw.
int enqueue_dense_reduce(double* A, long long lda, int n, const DenseWork& dw, void* stream);

}  // namespace tde
