"""First and last eigenvector rows at the top merge (tde_eigvals_rows), through
the C-ABI, against the oracle (LAPACK eigenvectors) and the Gauss-Legendre
closed form (Golub-Welsch weights 2 q_0k^2 of the Legendre Jacobi matrix).

Rows are compared entrywise (absolute error of unit-vector entries, 1e-10
plus 64 eps ||T|| / gap_k, the conditioning of an eigenvector; |q_0k|,
|q_(n-1)k| and their product, which do not depend on a column's sign); the W+
family, whose eigenvalue pairs agree to
below 1e-16 relative, has no individual rows to compare and is left out.
"""
import numpy as np
import pytest

import oracle
import tdgen

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _step(msg):
    print(f"[gpu-rows] {msg}", flush=True)


@pytest.fixture(scope="module")
def tde():
    import torch

    import paper_2605_26599_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def _gaps(lam):
    """Distance of every eigenvalue to its nearest neighbour (inf for n = 1)."""
    g = np.full(len(lam), np.inf)
    if len(lam) > 1:
        dl = np.diff(lam)
        g[:-1] = dl
        g[1:] = np.minimum(g[1:], dl)
    return g


def _rows(tde, d, e, leaf=None, offsets=None):
    lam, q0, q1 = tde.eigvals_rows(_t(d), _t(e if len(e) else np.zeros(1)), offsets=offsets, leaf=leaf)
    return lam.cpu().numpy(), q0.cpu().numpy(), q1.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 5, 31, 64, 100, 1000])
@pytest.mark.parametrize("leaf", [1, 8, 32])
def test_gauss_legendre(tde, n, leaf):
    _step(f"Gauss-Legendre n={n} leaf={leaf}")
    k = np.arange(1, n, dtype=np.float64)
    e = k / np.sqrt(4.0 * k * k - 1.0)
    lam, q0, q1 = _rows(tde, np.zeros(n), e, leaf=leaf)
    x, wgt = np.polynomial.legendre.leggauss(n)
    assert np.abs(lam - x).max() <= 1e-13
    assert np.all(q0 >= 0)
    assert np.abs(2.0 * q0 * q0 - wgt).max() <= 1e-12
    # exact for polynomials of degree <= 2n - 1
    for deg in sorted({dg for dg in (0, 1, 2, 2 * n - 2, 2 * n - 1) if 0 <= dg <= 2 * n - 1}):
        quad = float(np.dot(2.0 * q0 * q0, lam ** deg))
        exact = (2.0 / (deg + 1)) if deg % 2 == 0 else 0.0
        assert abs(quad - exact) <= 1e-11 * max(1.0, abs(exact))


@pytest.mark.parametrize("fam", ["uniform", "normal", "toeplitz", "clustered"])
@pytest.mark.parametrize("leaf", [1, 4, 32])
def test_rows_match_oracle(tde, fam, leaf):
    for n in [2, 3, 17, 200, 1000, 4097]:
        _step(f"rows fam={fam} leaf={leaf} n={n}")
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
        lam, q0, q1 = _rows(tde, d, e, leaf=leaf)
        lr, r0, r1 = oracle.boundary_rows(d, e)
        assert np.abs(lam - lr).max() <= 2e-11 * tdgen.tnorm1(d, e)
        assert np.all(q0 >= 0)
        # a column's sign is fixed by q_0k >= 0, which is decided by rounding
        # when q_0k is negligible (eigenvectors localised away from row 0), so
        # compare what does not depend on it
        # an eigenvector is determined only to about eps ||T|| / gap_k
        tol = TOL + 64.0 * np.finfo(float).eps * tdgen.tnorm1(d, e) / _gaps(lr)
        assert np.all(np.abs(q0 - np.abs(r0)) <= tol), np.max(np.abs(q0 - np.abs(r0)) / tol)
        assert np.all(np.abs(np.abs(q1) - np.abs(r1)) <= tol), np.max(np.abs(np.abs(q1) - np.abs(r1)) / tol)
        assert np.all(np.abs(q0 * q1 - r0 * r1) <= tol), np.max(np.abs(q0 * q1 - r0 * r1) / tol)
        assert abs(np.sum(q0 * q0) - 1.0) <= 1e-12 and abs(np.sum(q1 * q1) - 1.0) <= 1e-12


@pytest.mark.parametrize("wide_min", [None, 1 << 30])
def test_rows_with_fuse_few(tde, wide_min):
    """Rows with the fused limit lowered on levels of few merges (the larger
    merges' roots, z-hat and rows then come from the root-parallel kernels:
    the wide sweeps, or with wide_min 2^30 the regular tiles) match the
    oracle as in the default setting."""
    tde.set_defaults(fuse_few=32, wide_min=wide_min)
    try:
        for fam, n in [("uniform", 4097), ("toeplitz", 1000), ("clustered", 4097), ("normal", 3000)]:
            _step(f"rows fuse_few=32 wide_min={wide_min} fam={fam} n={n}")
            d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
            lam, q0, q1 = _rows(tde, d, e, leaf=32)
            lr, r0, r1 = oracle.boundary_rows(d, e)
            assert np.abs(lam - lr).max() <= 2e-11 * tdgen.tnorm1(d, e)
            tol = TOL + 64.0 * np.finfo(float).eps * tdgen.tnorm1(d, e) / _gaps(lr)
            assert np.all(np.abs(q0 - np.abs(r0)) <= tol)
            assert np.all(np.abs(np.abs(q1) - np.abs(r1)) <= tol)
            assert np.all(np.abs(q0 * q1 - r0 * r1) <= tol)
    finally:
        tde.set_defaults()


def test_rows_batched_matches_single(tde):
    sizes = [0, 1, 2, 3, 70, 500, 1025]
    probs = [tdgen.tridiag("uniform", s, cfg=tdgen.CFG_TEST, inst=i) for i, s in enumerate(sizes)]
    bt = tdgen.pack(probs)
    offs = [int(x) for x in bt.offsets]
    lam, q0, q1 = _rows(tde, bt.d, bt.e, offsets=offs)
    for b, (d, e) in enumerate(probs):
        s, t = offs[b], offs[b + 1]
        if t == s:
            continue
        _step(f"batched rows problem {b} n={t - s}")
        l1, a0, a1 = _rows(tde, d, e)
        assert np.array_equal(lam[s:t], l1) and np.array_equal(q0[s:t], a0) and np.array_equal(q1[s:t], a1)


def test_rows_do_not_change_eigenvalues(tde):
    """Rows mode computes the same eigenvalues, bit for bit, as the plain solve."""
    for fam, n in [("uniform", 20000), ("toeplitz", 3000)]:
        d, e = tdgen.tridiag(fam, n)
        lam, _, _ = _rows(tde, d, e)
        plain = tde.eigvals(_t(d), _t(e)).cpu().numpy()
        assert np.array_equal(lam, plain)
