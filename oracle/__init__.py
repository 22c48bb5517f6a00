"""ORACLE -- test infrastructure only.

Plain, slow CPU implementations of what the GPU path computes, used to judge it.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

* ``eigvals`` / ``eigvals_index`` / ``counts`` -- FP64 Sturm-sequence bisection
  (``sturm.c``): the spectrum of T, which the paper's correctness theorem
  (Section 3.2) says boundary-row D&C returns.
* ``ql_eigvals`` -- plain implicit-QL eigenvalues (``ql.c``), the sequential
  QR/QL baseline the paper compares against (Sections 2.1, 5.2).
* ``exact_charpoly_roots`` -- brute force for tiny n: exact rational
  characteristic polynomial of the dense matrix (Faddeev-LeVerrier), roots by
  ``mpmath.polyroots`` at 60+ digits.  Pins the bisection oracle.
* ``householder_tridiagonal`` / ``dense_eigvals`` -- textbook Householder
  reduction of a dense symmetric matrix to tridiagonal form (the reduction
  phase of dense EVD, Section 2.1), then bisection.
* ``grad_reference`` -- dense Hellmann-Feynman gradient of L = sum_k w_k lambda_k:
  dL/dd_i = sum_k w_k q_ik^2, dL/de_i = sum_k 2 w_k q_ik q_(i+1)k, with Q from
  LAPACK (``scipy.linalg.eigh_tridiagonal``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile sturm.c and ql.c into liboracle.so (plain -O2, IEEE semantics kept)."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, "sturm.c"), os.path.join(_HERE, "ql.c")]
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
               "-ffp-contract=off", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        lib.oracle_eigvals.argtypes = [i64, dp, dp, dp]
        lib.oracle_eigvals.restype = ctypes.c_int
        lib.oracle_eigvals_index.argtypes = [i64, dp, dp, i64, ip, dp]
        lib.oracle_eigvals_index.restype = ctypes.c_int
        lib.oracle_counts.argtypes = [i64, dp, dp, i64, dp, ip]
        lib.oracle_counts.restype = ctypes.c_int
        lib.oracle_counts_scalar.argtypes = [i64, dp, dp, i64, dp, ip]
        lib.oracle_counts_scalar.restype = ctypes.c_int
        lib.ql_eigvals.argtypes = [i64, dp, dp, dp]
        lib.ql_eigvals.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _prep(d, e):
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.size
    e = np.ascontiguousarray(e, dtype=np.float64)
    if e.size < max(n - 1, 0):
        raise ValueError("e must hold n-1 entries")
    if e.size == 0:
        e = np.zeros(1)
    return d, e, n


def _check(rc):
    if rc == -1:
        raise ValueError("non-finite input")
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    if rc == -3:
        raise ValueError("bad argument")
    if rc != 0:
        raise RuntimeError(f"oracle status {rc}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def eigvals(d, e) -> np.ndarray:
    """All eigenvalues of T(d, e), ascending, by Sturm bisection."""
    d, e, n = _prep(d, e)
    out = np.empty(n, dtype=np.float64)
    if n:
        _check(_load().oracle_eigvals(n, _dp(d), _dp(e), _dp(out)))
    return out


def eigvals_index(d, e, ks) -> np.ndarray:
    """lambda_k for each 0-based k in ks (ascending spectrum order)."""
    d, e, n = _prep(d, e)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    out = np.empty(ks.size, dtype=np.float64)
    if ks.size:
        _check(_load().oracle_eigvals_index(n, _dp(d), _dp(e), ks.size, _ip(ks), _dp(out)))
    return out


def counts(d, e, x) -> np.ndarray:
    """#{eigenvalues < x_j} for every point x_j."""
    d, e, n = _prep(d, e)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.size, dtype=np.int64)
    if x.size:
        _check(_load().oracle_counts(n, _dp(d), _dp(e), x.size, _dp(x), _ip(out)))
    return out


def counts_scalar(d, e, x) -> np.ndarray:
    """As counts, one point at a time (checks the grouped evaluation)."""
    d, e, n = _prep(d, e)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.size, dtype=np.int64)
    if x.size:
        _check(_load().oracle_counts_scalar(n, _dp(d), _dp(e), x.size, _dp(x), _ip(out)))
    return out


def certify(d, e, mu, t) -> int:
    """Number of indices k for which the Sturm counts fail to certify
    |mu_k - lambda_k| <= t, i.e. not (count(mu_k - t) <= k < count(mu_k + t)).
    0 means every computed eigenvalue is within t of the true k-th eigenvalue."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n = mu.size
    lo = counts(d, e, mu - t)
    hi = counts(d, e, mu + t)
    k = np.arange(n)
    bad = (lo > k) | (hi <= k)
    return int(bad.sum())


def ql_eigvals(d, e) -> np.ndarray:
    d, e, n = _prep(d, e)
    out = np.empty(n, dtype=np.float64)
    if n:
        rc = _load().ql_eigvals(n, _dp(d), _dp(e), _dp(out))
        if rc == 1:
            raise RuntimeError("QL did not converge")
        _check(rc)
    return out


# ----------------------------------------------------------------------------
# Brute force for tiny n (pins the bisection oracle independently of the
# tridiagonal recurrence it uses).
# ----------------------------------------------------------------------------

def _dense_fraction(d, e):
    n = len(d)
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        A[i][i] = Fraction(float(d[i]))
    for i in range(n - 1):
        A[i][i + 1] = Fraction(float(e[i]))
        A[i + 1][i] = Fraction(float(e[i]))
    return A


def charpoly_fraction(d, e):
    """Exact coefficients c[0..n] of det(x I - A), A = T(d, e) built as a dense
    rational matrix from the binary64 inputs, by the Faddeev-LeVerrier recursion
    M_1 = I, c_{n-1} = -tr(A); M_k = A M_{k-1} + c_{n-k+1} I, c_{n-k} = -tr(A M_k)/k."""
    A = _dense_fraction(d, e)
    n = len(A)
    c = [Fraction(0)] * (n + 1)
    c[n] = Fraction(1)
    M = [[Fraction(0)] * n for _ in range(n)]
    for k in range(1, n + 1):
        # M <- A M + c_{n-k+1} I
        AM = [[sum(A[i][t] * M[t][j] for t in range(n)) for j in range(n)] for i in range(n)]
        for i in range(n):
            AM[i][i] += c[n - k + 1]
        M = AM
        AMk = [[sum(A[i][t] * M[t][j] for t in range(n)) for j in range(n)] for i in range(n)]
        c[n - k] = -sum(AMk[i][i] for i in range(n)) / k
    return c


def exact_charpoly_roots(d, e, dps: int = 80):
    """Eigenvalues of tiny T as high-precision mpmath numbers (sorted)."""
    import mpmath

    c = charpoly_fraction(d, e)
    n = len(c) - 1
    if n == 0:
        return []
    with mpmath.workdps(dps):
        coeffs = [mpmath.mpf(c[k].numerator) / mpmath.mpf(c[k].denominator) for k in range(n, -1, -1)]
        roots = mpmath.polyroots(coeffs, maxsteps=2000, extraprec=4 * dps)
        re = sorted(mpmath.re(r) for r in roots)
    return re


# ----------------------------------------------------------------------------
# Gradient reference (dense eigenvectors from LAPACK).
# ----------------------------------------------------------------------------

def grad_reference(d, e, w):
    """Dense Hellmann-Feynman gradient of L = sum_k w_k lambda_k(T):
    g_d[i] = sum_k w_k q_ik^2 and g_e[i] = sum_k 2 w_k q_ik q_(i+1)k, where the
    columns q_k of Q are the unit eigenvectors of T in ascending eigenvalue order."""
    from scipy.linalg import eigh_tridiagonal

    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    lam, Q = eigh_tridiagonal(d, e, lapack_driver="stemr")
    Qw = Q * w[None, :]
    gd = np.einsum("ik,ik->i", Qw, Q)
    ge = 2.0 * np.einsum("ik,ik->i", Qw[:-1], Q[1:])
    return lam, gd, ge


def boundary_rows(d, e):
    """Eigenvalues and the first and last rows of the eigenvector matrix of T
    (the rows the method propagates, Section 3.2), from LAPACK eigenvectors
    (scipy.linalg.eigh_tridiagonal): returns (lam, q0, qlast) in ascending
    eigenvalue order, each column signed so that q0_k >= 0 (qlast_k >= 0 when
    q0_k = 0)."""
    from scipy.linalg import eigh_tridiagonal

    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    if len(d) == 0:
        z = np.zeros(0)
        return z, z, z
    if len(d) == 1:
        return d.copy(), np.ones(1), np.ones(1)
    lam, Q = eigh_tridiagonal(d, e, lapack_driver="stemr")
    q0, q1 = Q[0].copy(), Q[-1].copy()
    sg = np.where((q0 < 0) | ((q0 == 0) & (q1 < 0)), -1.0, 1.0)
    return lam, q0 * sg, q1 * sg


def selected_rows(d, e, rows):
    """Eigenvalues and the requested rows of the eigenvector matrix of T
    (Algorithm 1's requested rows sigma; Lemma 2: the rows of Q S are the
    requested rows of Q times S), from LAPACK eigenvectors
    (scipy.linalg.eigh_tridiagonal): returns (lam, Qs) with Qs[i, k] = q_(rows[i]) k
    for ascending lam, rows in the order given (repeats allowed), each column
    signed so that q_0k >= 0 (q_(n-1)k >= 0 when q_0k = 0) -- the convention of
    boundary_rows."""
    from scipy.linalg import eigh_tridiagonal

    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    n = len(d)
    if n == 0:
        return np.zeros(0), np.zeros((len(rows), 0))
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    if n == 1:
        return d.copy(), np.ones((len(rows), 1))
    lam, Q = eigh_tridiagonal(d, e, lapack_driver="stemr")
    sg = np.where((Q[0] < 0) | ((Q[0] == 0) & (Q[-1] < 0)), -1.0, 1.0)
    return lam, Q[rows] * sg[None, :]


def row_weights_interlacing(d, e, r):
    """Squares q_rk^2 of row r of the eigenvector matrix from eigenvalues alone:
    q_rk^2 = prod_j (lambda_k - mu_j) prod_j (lambda_k - nu_j) / prod_(j != k) (lambda_k - lambda_j),
    with mu the spectrum of T[0:r, 0:r] and nu that of T[r+1:, r+1:] (the
    classical identity for the diagonal of the resolvent of a tridiagonal:
    (T - x)^-1_rr = chi_(0..r-1)(x) chi_(r+1..n-1)(x) / chi(x)).  Every
    spectrum comes from bisection (eigvals); products run as chains of ratios
    so they neither overflow nor underflow.  For small n only (O(n^2))."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = len(d)
    lam = eigvals(d, e)
    mu = eigvals(d[:r], e[:max(r - 1, 0)]) if r > 0 else np.zeros(0)
    nu = eigvals(d[r + 1:], e[r + 1:]) if r + 1 < n else np.zeros(0)
    out = np.empty(n)
    for k in range(n):
        others = np.delete(lam, k)
        num = np.concatenate([mu, nu])
        # n - 1 numerator and n - 1 denominator factors, paired in sorted order
        ratio = 1.0
        for a, b in zip(np.sort(num), np.sort(others)):
            ratio *= (lam[k] - a) / (lam[k] - b)
        out[k] = ratio
    return out


# ----------------------------------------------------------------------------
# Dense front end: reduction of a symmetric matrix to tridiagonal form.
# ----------------------------------------------------------------------------

def householder_tridiagonal(A):
    """Orthogonal reduction of a real symmetric A to tridiagonal T = H^T A H
    (the reduction phase of dense symmetric EVD, Section 2.1: the eigenvalues
    of T are those of A).  Textbook Householder reduction in FP64, one
    reflector per column: for column k, H_k = I - beta v v^T maps A[k+1:, k]
    onto a multiple of e_1 and is applied from both sides to the trailing
    block (p = beta B v, w = p - (beta/2)(p^T v) v, B <- B - v w^T - w v^T).
    Returns (d, e): the diagonal and subdiagonal of T."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    for k in range(n - 2):
        x = A[k + 1:, k].copy()
        nx = np.linalg.norm(x)
        if nx == 0.0:
            continue
        alpha = -nx if x[0] >= 0.0 else nx
        v = x
        v[0] -= alpha
        vv = float(v @ v)
        if vv == 0.0:
            continue
        beta = 2.0 / vv
        B = A[k + 1:, k + 1:]
        p = beta * (B @ v)
        w = p - (0.5 * beta * float(p @ v)) * v
        B -= np.outer(v, w) + np.outer(w, v)
        A[k + 1:, k] = 0.0
        A[k, k + 1:] = 0.0
        A[k + 1, k] = alpha
        A[k, k + 1] = alpha
    return np.diag(A).copy(), np.diag(A, -1).copy()


def dense_eigvals(A):
    """Eigenvalues (ascending) of a dense real symmetric A: Householder
    reduction to tridiagonal form, then Sturm bisection (eigvals)."""
    d, e = householder_tridiagonal(A)
    return eigvals(d, e)
