"""Pins for the CPU oracle (Sturm bisection), against facts fixed by mathematics
rather than by the oracle itself: closed forms, invariants, exact rational brute
force, an independent dense high-precision eigensolver, and special cases.

Each pin is chosen so that a plausible slip in the oracle (a dropped square on
e, a shifted index in the pivot recurrence, a wrong comparison in the bisection
update, a lost scale factor) fails at least one test.
"""
import math

import numpy as np
import pytest

import oracle
import tdgen

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _err(a, b, d, e):
    diff = np.abs(np.asarray(a) - np.asarray(b)).max()
    tn = tdgen.tnorm1(d, e)
    if tn == 0.0:
        return 0.0 if diff == 0.0 else np.inf
    return diff / (tn * EPS)


# --- closed form -------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 17, 64, 257, 1000])
@pytest.mark.parametrize("a,b", [(2.0, -1.0), (2.0, 0.25), (-0.5, 3.0), (0.0, 1e-3)])
def test_toeplitz_closed_form(n, a, b):
    # Eigenvalues of the Toeplitz tridiagonal (d = a, e = b): a + 2 b cos(k pi/(n+1)), k = 1..n.
    import mpmath

    d = np.full(n, a)
    e = np.full(n - 1, b)
    with mpmath.workdps(40):
        exact = np.sort([float(a + 2 * mpmath.mpf(b) * mpmath.cos(k * mpmath.pi / (n + 1)))
                         for k in range(1, n + 1)])
    assert np.abs(oracle.eigvals(d, e) - exact).max() <= 4.0 * EPS * (abs(a) + 2 * abs(b))


# --- invariants --------------------------------------------------------------

@pytest.mark.parametrize("fam", ["uniform", "normal", "wilkinson", "clustered", "paper_normal"])
def test_trace_and_frobenius(fam):
    n = 700
    d, e = tdgen.tridiag(fam, n)
    lam = oracle.eigvals(d, e)
    tn = tdgen.tnorm1(d, e)
    # trace(T) = sum d_i = sum lambda_k
    assert abs(math.fsum(lam) - math.fsum(d)) <= n * 4 * EPS * tn
    # ||T||_F^2 = sum d_i^2 + 2 sum e_i^2 = sum lambda_k^2
    fro = math.fsum(d * d) + 2.0 * math.fsum(e * e)
    assert abs(math.fsum(lam * lam) - fro) <= 2 * n * tn * 4 * EPS * tn
    # ascending, and inside the Gershgorin discs' hull
    assert np.all(np.diff(lam) >= 0)
    assert lam[0] >= -tn and lam[-1] <= tn


# --- exact brute force -------------------------------------------------------

@pytest.mark.parametrize("n", range(1, 9))
@pytest.mark.parametrize("fam", ["uniform", "normal", "wilkinson", "clustered"])
def test_exact_charpoly_tiny(n, fam):
    for inst in range(3):
        d, e = tdgen.tridiag(fam, n, inst=inst)
        exact = np.array([float(x) for x in oracle.exact_charpoly_roots(d, e)])
        assert _err(oracle.eigvals(d, e), exact, d, e) <= 4.0


def test_wilkinson21_exact():
    # W+_21: d_i = |i - 10|, e = 1.  Its top eigenvalues come in pairs that agree
    # to about 14 digits, a classic stress case for any eigensolver.
    d, e = tdgen.tridiag("wilkinson", 21)
    exact = np.array([float(x) for x in oracle.exact_charpoly_roots(d, e, dps=100)])
    got = oracle.eigvals(d, e)
    assert _err(got, exact, d, e) <= 4.0
    assert abs(exact[-1] - 10.746194182903393) < 1e-12  # largest eigenvalue of W+_21


def test_golden_exact_small():
    # Stored exact eigenvalues (tests/golden/make_exact_small.py): the oracle's
    # bisection within a few ulps of ||T||, and facts that pin the fixture itself.
    from conftest import load_exact_small

    cases = {name: (d, e, lam) for name, d, e, lam in load_exact_small()}
    assert len(cases) >= 10
    for name, (d, e, lam) in cases.items():
        assert np.all(np.diff(lam) >= 0), name
        assert _err(oracle.eigvals(d, e), lam, d, e) <= 4.0, name
        assert abs(lam.sum() - d.sum()) <= 1e-12 * max(1.0, np.abs(d).sum()), name  # trace
    assert cases["wilkinson_plus_21"][2][-1] == 10.746194182903393  # largest eigenvalue of W+_21
    wm = cases["wilkinson_minus_21"][2]
    assert np.array_equal(wm, -wm[::-1]) and wm[10] == 0.0  # W-_21 is similar to -W-_21
    k = np.arange(1, 17)
    assert np.abs(cases["toeplitz_121_n16"][2] - (2 - 2 * np.cos(k * np.pi / 17))).max() <= 8 * EPS
    d, e, lam = cases["n2"]
    m, r = 0.5 * (d[0] + d[1]), math.hypot(0.5 * (d[0] - d[1]), e[0])
    assert np.abs(lam - [m - r, m + r]).max() <= 4 * EPS


@pytest.mark.parametrize("fam", ["uniform", "wilkinson", "paper_clustered"])
def test_dense_high_precision(fam):
    # An independent dense symmetric eigensolver (mpmath Jacobi, 40 digits).
    import mpmath

    n = 48
    d, e = tdgen.tridiag(fam, n, inst=7)
    with mpmath.workdps(40):
        A = mpmath.matrix(n, n)
        for i in range(n):
            A[i, i] = d[i]
        for i in range(n - 1):
            A[i, i + 1] = e[i]
            A[i + 1, i] = e[i]
        ev = mpmath.eigsy(A, eigvals_only=True)
        exact = np.array(sorted(float(x) for x in ev))
    assert _err(oracle.eigvals(d, e), exact, d, e) <= 4.0


def test_library_crosscheck():
    # LAPACK's bisection (dstebz) through scipy: an independent implementation.
    from scipy.linalg import eigvalsh_tridiagonal

    for fam in ["uniform", "normal", "wilkinson", "clustered"]:
        d, e = tdgen.tridiag(fam, 1500)
        ref = eigvalsh_tridiagonal(d, e, lapack_driver="stebz")
        assert _err(oracle.eigvals(d, e), ref, d, e) <= 8.0


# --- special cases -------------------------------------------------------------

def test_n1_and_n0():
    for v in [3.25, -1e-7, 6.0e12]:
        assert abs(oracle.eigvals(np.array([v]), np.zeros(0))[0] - v) <= 2 * EPS * abs(v)
    assert oracle.eigvals(np.array([0.0]), np.zeros(0))[0] == 0.0
    assert oracle.eigvals(np.zeros(0), np.zeros(0)).size == 0


def test_n2_closed_form():
    g = tdgen.rng(tdgen.CFG_TEST, 0, 2, 0)
    for _ in range(50):
        d = g.uniform(-3, 3, 2)
        e = g.uniform(-3, 3, 1)
        m = 0.5 * (d[0] + d[1])
        r = math.hypot(0.5 * (d[0] - d[1]), e[0])
        assert _err(oracle.eigvals(d, e), [m - r, m + r], d, e) <= 4.0


def test_diagonal_gives_sorted_d():
    d, _ = tdgen.tridiag("normal", 300)
    lam = oracle.eigvals(d, np.zeros(299))
    assert np.all(np.abs(lam - np.sort(d)) <= 2 * EPS * np.abs(np.sort(d)) + 1e-300)


def test_scale_and_shift_equivariance():
    d, e = tdgen.tridiag("uniform", 400)
    lam = oracle.eigvals(d, e)
    # alpha a power of two: scaling is exact, so the result scales bitwise.
    for alpha in [2.0**-30, 0.5, 8.0, 2.0**40]:
        assert np.array_equal(oracle.eigvals(alpha * d, alpha * e), alpha * lam)
    beta = 0.375
    assert _err(oracle.eigvals(d + beta, e), lam + beta, d, e) <= 4.0


def test_sign_and_reversal_invariance():
    d, e = tdgen.tridiag("normal", 333)
    lam = oracle.eigvals(d, e)
    # flipping off-diagonal signs is a diagonal similarity; the recurrence sees only e^2
    assert np.array_equal(oracle.eigvals(d, -e), lam)
    # reversing the index order is a permutation similarity (different pivots, same spectrum)
    assert _err(oracle.eigvals(d[::-1].copy(), e[::-1].copy()), lam, d, e) <= 4.0


def test_direct_sum():
    d1, e1 = tdgen.tridiag("uniform", 37, inst=1)
    d2, e2 = tdgen.tridiag("uniform", 51, inst=2)
    d = np.concatenate([d1, d2])
    e = np.concatenate([e1, [0.0], e2])
    both = np.sort(np.concatenate([oracle.eigvals(d1, e1), oracle.eigvals(d2, e2)]))
    assert _err(oracle.eigvals(d, e), both, d, e) <= 4.0


def test_nonfinite_rejected():
    d = np.array([1.0, np.nan, 2.0])
    with pytest.raises(ValueError):
        oracle.eigvals(d, np.zeros(2))
    with pytest.raises(ValueError):
        oracle.eigvals(np.ones(3), np.array([np.inf, 0.0]))


# --- the index / count entry points ------------------------------------------

def test_index_matches_full_and_certify():
    d, e = tdgen.tridiag("uniform", 900)
    lam = oracle.eigvals(d, e)
    ks = np.array([0, 1, 17, 450, 898, 899])
    assert np.array_equal(oracle.eigvals_index(d, e, ks), lam[ks])
    t = 8 * EPS * tdgen.tnorm1(d, e)
    assert oracle.certify(d, e, lam, t) == 0
    bad = lam.copy()
    bad[123] += 1e-9  # a planted error far above t must be caught
    assert oracle.certify(d, e, bad, t) >= 1
    c = oracle.counts(d, e, np.array([-1e9, 1e9, 0.5 * (lam[10] + lam[11])]))
    assert list(c) == [0, 900, 11]


def test_grouped_counts_equal_scalar_counts():
    """The grouped Sturm counts (eight points sharing one loop) return exactly
    the one-point-at-a-time counts, at every point, including points on and
    next to eigenvalues, tails of the group and an empty group."""
    for fam, n in [("uniform", 1000), ("clustered", 777), ("wilkinson", 21), ("toeplitz", 64)]:
        d, e = tdgen.tridiag(fam, n)
        lam = oracle.eigvals(d, e)
        g = np.random.default_rng(n)
        x = np.concatenate([lam, np.nextafter(lam, np.inf), np.nextafter(lam, -np.inf),
                            g.uniform(lam[0] - 1, lam[-1] + 1, 1003)])
        for m in (x.size, 7, 8, 9, 1):
            assert np.array_equal(oracle.counts(d, e, x[:m]), oracle.counts_scalar(d, e, x[:m])), (fam, m)
        c = oracle.counts(d, e, np.sort(x))
        assert np.all(np.diff(c) >= 0) and c[0] >= 0 and c[-1] <= n


def test_ql_baseline_agrees():
    for fam in ["uniform", "toeplitz", "wilkinson", "clustered"]:
        d, e = tdgen.tridiag(fam, 600)
        assert _err(oracle.ql_eigvals(d, e), oracle.eigvals(d, e), d, e) <= 200.0


# --- gradient reference (dense Hellmann-Feynman) ----------------------------

def test_grad_reference_invariants_and_fd():
    n = 64
    d, e = tdgen.tridiag("uniform", n, cfg=tdgen.CFG_GRAD)
    w = tdgen.loss_weights(n)
    lam, gd, ge = oracle.grad_reference(d, e, w)
    L = float(np.dot(w, lam))
    gmax = max(np.abs(gd).max(), np.abs(ge).max())
    # columns of Q are unit vectors: sum_i g_d,i = sum_k w_k
    assert abs(gd.sum() - w.sum()) <= 1e-12 * np.abs(w).sum()
    # lambda(alpha T) = alpha lambda(T): d . g_d + e . g_e = L
    assert abs(np.dot(d, gd) + np.dot(e, ge) - L) <= 1e-12 * np.abs(w).sum() * tdgen.tnorm1(d, e)
    # coordinate-wise central differences of the bisection oracle
    h = 1e-6
    for i in [0, 5, 31, 63]:
        dp, dm = d.copy(), d.copy()
        dp[i] += h
        dm[i] -= h
        fd = (np.dot(w, oracle.eigvals(dp, e)) - np.dot(w, oracle.eigvals(dm, e))) / (2 * h)
        assert abs(fd - gd[i]) <= 1e-7 * gmax
    for i in [0, 17, 62]:
        ep, em = e.copy(), e.copy()
        ep[i] += h
        em[i] -= h
        fd = (np.dot(w, oracle.eigvals(d, ep)) - np.dot(w, oracle.eigvals(d, em))) / (2 * h)
        assert abs(fd - ge[i]) <= 1e-7 * gmax


# --- boundary rows (first and last eigenvector rows) -------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 8, 40, 200])
def test_boundary_rows_gauss_legendre(n):
    """Golub-Welsch: for the Legendre Jacobi matrix (d = 0, e_k = k/sqrt(4k^2-1))
    the eigenvalues are the Gauss-Legendre nodes and 2 q_0k^2 the weights."""
    k = np.arange(1, n, dtype=np.float64)
    e = k / np.sqrt(4.0 * k * k - 1.0)
    lam, q0, q1 = oracle.boundary_rows(np.zeros(n), e)
    x, wgt = np.polynomial.legendre.leggauss(n)
    assert np.abs(lam - x).max() <= 1e-13
    assert np.abs(2.0 * q0 * q0 - wgt).max() <= 1e-13
    assert np.all(q0 >= 0)
    assert abs(np.sum(q1 * q1) - 1.0) <= 1e-13


def test_boundary_rows_identities():
    """Unit rows, orthogonal rows, and the resolvent identity
    q_0k q_(n-1)k = prod(e) / prod_{j != k} (lambda_k - lambda_j)."""
    for fam, n in [("uniform", 7), ("normal", 10), ("toeplitz", 12), ("clustered", 9)]:
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
        lam, q0, q1 = oracle.boundary_rows(d, e)
        assert abs(np.sum(q0 * q0) - 1.0) <= 1e-14 and abs(np.sum(q1 * q1) - 1.0) <= 1e-14
        assert abs(np.sum(q0 * q1)) <= 1e-14
        pe = np.prod(e)
        for kk in range(n):
            den = np.prod([lam[kk] - lam[j] for j in range(n) if j != kk])
            assert abs(q0[kk] * q1[kk] - pe / den) <= 1e-12 * max(1.0, abs(pe / den))


# --- requested rows (Algorithm 1 with an arbitrary row list) ------------------

@pytest.mark.parametrize("fam,n", [("uniform", 9), ("normal", 12), ("toeplitz", 10), ("clustered", 8),
                                   ("wilkinson", 7)])
def test_selected_rows_interlacing_identity(fam, n):
    """q_rk^2 of every row from eigenvalues alone (the resolvent-diagonal
    identity, through the bisection oracle's spectra of T and of the two
    blocks left when row and column r are removed)."""
    d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
    lam, Q = oracle.selected_rows(d, e, np.arange(n))
    assert np.abs(lam - oracle.eigvals(d, e)).max() <= 1e-14 * tdgen.tnorm1(d, e)
    for r in range(n):
        w = oracle.row_weights_interlacing(d, e, r)
        assert np.abs(w - Q[r] ** 2).max() <= 1e-12, r


@pytest.mark.parametrize("fam,n", [("uniform", 30), ("normal", 25), ("toeplitz", 16)])
def test_selected_rows_eigen_equation(fam, n):
    """All rows requested, shuffled and repeated: the distinct rows form an
    orthogonal Q with T Q = Q diag(lambda) (which fixes the relative signs of
    the rows), repeats equal their first occurrence, and every column is signed
    so that q_0k >= 0."""
    d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
    g = np.random.default_rng(5)
    perm = g.permutation(n)
    rows = np.concatenate([perm, perm[:7]])
    lam, Qs = oracle.selected_rows(d, e, rows)
    Q = np.empty((n, n))
    Q[perm] = Qs[:n]
    assert np.array_equal(Qs[n:], Qs[:7])
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13
    assert np.abs(T @ Q - Q * lam[None, :]).max() <= 1e-13 * tdgen.tnorm1(d, e)
    assert np.all((Q[0] > 0) | ((Q[0] == 0) & (Q[-1] >= 0)))


def test_selected_rows_boundary_and_gauss():
    """Rows {0, n-1} agree with boundary_rows; row 0 of the Legendre Jacobi
    matrix gives the Gauss-Legendre weights (Golub-Welsch)."""
    d, e = tdgen.tridiag("uniform", 40, cfg=tdgen.CFG_TEST)
    lam, q0, q1 = oracle.boundary_rows(d, e)
    lam2, Qs = oracle.selected_rows(d, e, [39, 0])
    assert np.array_equal(lam, lam2) and np.array_equal(Qs[1], q0) and np.array_equal(Qs[0], q1)
    n = 24
    k = np.arange(1, n, dtype=np.float64)
    _, Qs = oracle.selected_rows(np.zeros(n), k / np.sqrt(4.0 * k * k - 1.0), [0])
    _, wgt = np.polynomial.legendre.leggauss(n)
    assert np.abs(2.0 * Qs[0] ** 2 - wgt).max() <= 1e-13


# --- dense front end (reduction to tridiagonal form) --------------------------

def _prescribed(n, seed, spread=1.0):
    g = np.random.default_rng(seed)
    Q, R = np.linalg.qr(g.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))[None, :]
    lam = np.sort(g.uniform(-spread, spread, n))
    return Q @ np.diag(lam) @ Q.T, lam


@pytest.mark.parametrize("n", [3, 5, 40, 200])
def test_dense_reduction_prescribed_spectrum(n):
    """A = Q diag(lambda) Q^T with a random orthogonal Q: the reduced
    tridiagonal has exactly the prescribed eigenvalues (to the reduction's
    rounding), and trace and Frobenius norm are kept."""
    A, lam = _prescribed(n, 7 + n)
    A = 0.5 * (A + A.T)
    d, e = oracle.householder_tridiagonal(A)
    assert d.shape == (n,) and e.shape == (n - 1,)
    got = oracle.eigvals(d, e)
    assert np.abs(got - lam).max() <= 64 * n * np.finfo(float).eps * np.abs(lam).max()
    assert abs(d.sum() - np.trace(A)) <= 1e-12 * n
    assert abs((d @ d + 2 * e @ e) - np.sum(A * A)) <= 1e-12 * np.sum(A * A)


def test_dense_reduction_special_cases():
    """A tridiagonal input stays tridiagonal up to the signs of e; n = 1, 2
    need no reflector; 2 J - I (J the 3 x 3 all-ones matrix) has eigenvalues
    5, -1, -1."""
    d0, e0 = tdgen.tridiag("uniform", 30, cfg=tdgen.CFG_TEST)
    T = np.diag(d0) + np.diag(e0, 1) + np.diag(e0, -1)
    d, e = oracle.householder_tridiagonal(T)
    assert np.abs(d - d0).max() <= 1e-15 and np.abs(np.abs(e) - np.abs(e0)).max() <= 1e-15
    d, e = oracle.householder_tridiagonal(np.array([[3.0]]))
    assert d.tolist() == [3.0] and e.size == 0
    d, e = oracle.householder_tridiagonal(np.array([[1.0, 2.0], [2.0, -1.0]]))
    assert d.tolist() == [1.0, -1.0] and e.tolist() == [2.0]
    A = 2.0 * np.ones((3, 3)) - np.eye(3)
    lam = oracle.dense_eigvals(A)
    assert np.abs(lam - np.array([-1.0, -1.0, 5.0])).max() <= 1e-14
