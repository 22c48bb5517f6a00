// Host-side check of libtde_host's solver under AddressSanitizer and UBSan:
// reads n, d[n], e[n-1] from stdin, solves with workspace arrays of exactly
// the queried sizes (heap blocks, so any overrun is reported), prints the
// status and the eigenvalues.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../../include/tde_host.h"

int main() {
    long long n = 0;
    if (scanf("%lld", &n) != 1 || n < 0) return 2;
    std::vector<double> d(n), e(n > 0 ? n - 1 : 0);
    for (auto& x : d)
        if (scanf("%lf", &x) != 1) return 2;
    for (auto& x : e)
        if (scanf("%lf", &x) != 1) return 2;
    int64_t lw = 0, liw = 0;
    if (tde_host_workspace(n, &lw, &liw) != TDE_HOST_OK) return 3;
    double* work = (double*)malloc(sizeof(double) * (lw > 0 ? lw : 1));
    int* iwork = (int*)malloc(sizeof(int) * (liw > 0 ? liw : 1));
    double* lam = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    const int st = tde_host_eigvals(d.data(), e.empty() ? nullptr : e.data(), n, lam, work, lw, iwork, liw, 1);
    printf("%d\n", st);
    for (long long i = 0; i < n; ++i) printf("%.17g\n", lam[i]);
    free(work);
    free(iwork);
    free(lam);
    return 0;
}
