"""Requested eigenvector rows (Algorithm 1 with an arbitrary row list sigma,
tde_eigvals_selrows) through the C-ABI, against the oracle's LAPACK rows.

Entries are compared after aligning each column's sign with the oracle's (the
convention q_0k >= 0 is decided by rounding where q_0k is negligible), to
1e-10 plus 64 eps ||T||_1 / gap_k (an eigenvector is determined only to about
eps ||T|| / gap_k).  Where q_0k is not negligible its sign is checked too.
At sizes the dense oracle cannot reach, three consecutive requested rows must
satisfy the eigen-equation of their middle row, e_(r-1) q_(r-1)k + d_r q_rk +
e_r q_(r+1)k = lambda_k q_rk, and rows {0, n-1} must equal the boundary rows
of tde_eigvals_rows bit for bit.
"""
import numpy as np
import pytest

import oracle
import tdgen

pytestmark = pytest.mark.gpu

TOL = 1e-10
EPS = np.finfo(float).eps


def _step(msg):
    print(f"[gpu-selrows] {msg}", flush=True)


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
    g = np.full(len(lam), np.inf)
    if len(lam) > 1:
        dl = np.diff(lam)
        g[:-1] = dl
        g[1:] = np.minimum(g[1:], dl)
    return g


def _sel(tde, d, e, rows, **kw):
    lam, Q = tde.eigvals_selrows(_t(d), _t(e if len(e) else np.zeros(1)), rows, **kw)
    return lam.cpu().numpy(), Q.cpu().numpy()


def _compare(d, e, rows, lam, Q):
    lr, Qr = oracle.selected_rows(d, e, rows)
    tn = tdgen.tnorm1(d, e)
    assert np.abs(lam - lr).max() <= 2e-11 * tn
    tol = TOL + 64.0 * EPS * tn / _gaps(lr)
    sg = np.where(np.einsum("ik,ik->k", Q, Qr) < 0, -1.0, 1.0)
    err = np.abs(Q * sg[None, :] - Qr) / tol[None, :]
    assert err.max() <= 1.0, (float(err.max()), np.unravel_index(np.argmax(err), err.shape))
    # the sign convention where it is decided by more than rounding
    r0 = [i for i, r in enumerate(rows) if r == 0]
    if r0:
        q0 = Q[r0[0]]
        firm = np.abs(Qr[r0[0]]) > tol
        assert np.all(q0[firm] > 0)
    # repeats are copies of their first occurrence
    for i, r in enumerate(rows):
        j = list(rows).index(r)
        assert np.array_equal(Q[i], Q[j])


@pytest.mark.parametrize("fam", ["uniform", "normal", "toeplitz", "clustered"])
@pytest.mark.parametrize("leaf", [1, 4, 32])
def test_selrows_match_oracle(tde, fam, leaf):
    g = np.random.default_rng(11)
    for n in [1, 2, 3, 17, 200, 1000, 4097]:
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
        if n <= 200:
            perm = list(g.permutation(n))
            rows = perm + perm[: min(5, n)]  # every row, shuffled, with repeats
        else:
            pick = list(g.choice(n, 7, replace=False))
            rows = [n - 1, pick[0], 0, n // 2] + pick[1:] + [pick[0], 0]
        _step(f"selrows fam={fam} leaf={leaf} n={n} m={len(rows)}")
        lam, Q = _sel(tde, d, e, rows, leaf=leaf)
        _compare(d, e, rows, lam, Q)


def test_selrows_with_fuse_few_tiles(tde):
    """Requested rows when the larger merges of few-merge levels take the
    regular tiles (fuse_few 32, no wide sweeps): those levels' columns are
    then placed by the root kernels themselves, with no assembly launch."""
    g = np.random.default_rng(5)
    tde.set_defaults(fuse_few=32, wide_min=1 << 30)
    try:
        for fam, n in [("uniform", 4097), ("normal", 3000), ("clustered", 2049), ("toeplitz", 1000)]:
            pick = list(g.choice(n, 6, replace=False))
            rows = [0, n - 1] + pick + [pick[0]]
            _step(f"selrows fuse_few=32 tiles fam={fam} n={n}")
            d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_TEST)
            lam, Q = _sel(tde, d, e, rows, leaf=32)
            _compare(d, e, rows, lam, Q)
    finally:
        tde.set_defaults()


def test_selrows_gauss_legendre(tde):
    n = 300
    k = np.arange(1, n, dtype=np.float64)
    e = k / np.sqrt(4.0 * k * k - 1.0)
    _step("Gauss-Legendre weights from row 0")
    lam, Q = _sel(tde, np.zeros(n), e, [0], leaf=8)
    x, wgt = np.polynomial.legendre.leggauss(n)
    assert np.abs(lam - x).max() <= 1e-13
    assert np.all(Q[0] >= 0)
    assert np.abs(2.0 * Q[0] ** 2 - wgt).max() <= 1e-12


@pytest.mark.parametrize("fam,n,leaf", [("uniform", 65536, 32), ("toeplitz", 16384, 8), ("normal", 40000, 16)])
def test_selrows_full_size_properties(tde, fam, n, leaf):
    """Three consecutive rows satisfy the middle row's eigen-equation; rows
    {0, n-1} are the boundary rows of tde_eigvals_rows bit for bit; the
    eigenvalues are those of the plain solve bit for bit."""
    d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_FAMILIES)
    r = n // 3
    rows = [r + 1, 0, r, n - 1, r - 1, r]
    _step(f"selrows full size fam={fam} n={n} leaf={leaf}")
    lam, Q = _sel(tde, d, e, rows, leaf=leaf)
    tn = tdgen.tnorm1(d, e)
    res = e[r - 1] * Q[4] + d[r] * Q[2] + e[r] * Q[0] - lam * Q[2]
    assert np.abs(res).max() <= 1e-11 * tn, float(np.abs(res).max())
    # rows of unit eigenvectors: |q| <= 1
    assert np.abs(Q).max() <= 1.0 + 1e-12
    lr, q0, q1 = tde.eigvals_rows(_t(d), _t(e), leaf=leaf)
    assert np.array_equal(lam, lr.cpu().numpy())
    assert np.array_equal(Q[1], q0.cpu().numpy()) and np.array_equal(Q[3], q1.cpu().numpy())
    plain = tde.eigvals(_t(d), _t(e), leaf=leaf).cpu().numpy()
    assert np.array_equal(lam, plain)
    assert oracle.certify(d, e, lam, 2e-11 * tn) == 0


def test_selrows_arguments(tde):
    d, e = tdgen.tridiag("uniform", 100)
    for bad in ([100], [-1], [0, 5, 200]):
        with pytest.raises(tde.TDEError) as ex:
            _sel(tde, d, e, bad)
        assert ex.value.code == tde.TDE_EINVAL
    lam, Q = _sel(tde, d, e, [])
    assert Q.shape == (0, 100)
    assert np.abs(lam - oracle.eigvals(d, e)).max() <= 2e-11 * tdgen.tnorm1(d, e)
