"""The allocation-free entry point (tde_eigvals_noalloc) against tde_eigvals.

Both run the same kernels under the same plan, so the eigenvalues must agree
bit for bit, and both must meet the oracle gate max|dlambda| <= 2e-11 ||T||_1.
Two calls in a row (the second smaller, so stale tables or workspace contents
of the first would show), a non-finite input reported through the status
output, and sizes beyond the fixed scratch array rejected with TDE_EINVAL.
"""
import numpy as np
import pytest

import oracle
import tdgen

pytestmark = pytest.mark.gpu

GATE = 2e-11


def _step(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


@pytest.fixture(scope="module")
def tde():
    import torch

    import paper_2605_26599_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


@pytest.mark.parametrize("kw", [{}, {"leaf": 32}, {"leaf": 64, "leaf_dc": True},
                                {"leaf": 64, "leaf_dc": True, "sweep_cols": 16, "wide_min": 64}])
def test_noalloc_matches_eigvals_two_calls(tde, kw):
    import torch

    status = torch.full((1,), -99, dtype=torch.int32, device="cuda:0")
    for fam, n in (("uniform", 65536), ("toeplitz", 5000)):
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_FAMILIES)
        dv, ev = _t(d), _t(e)
        _step(f"{fam} n={n} {kw}")
        lam_na = tde.eigvals_noalloc(dv, ev, status=status, **kw)
        torch.cuda.synchronize()
        assert int(status.item()) == tde.TDE_OK
        lam_ref = tde.eigvals(dv, ev, **kw)
        a, b = lam_na.cpu().numpy(), lam_ref.cpu().numpy()
        assert np.array_equal(a, b), float(np.abs(a - b).max())
        tol = GATE * tdgen.tnorm1(d, e)
        if n <= 5000:
            ref = oracle.eigvals(d, e)
            assert float(np.abs(a - ref).max()) <= tol
        else:
            ks = np.linspace(0, n - 1, 257).astype(np.int64)
            assert float(np.abs(a[ks] - oracle.eigvals_index(d, e, ks)).max()) <= tol
            assert oracle.certify(d, e, a, tol) == 0


def test_noalloc_fuse_few(tde):
    """The fused limit on levels of few merges reaches the allocation-free
    plan too: two calls in a row (the second smaller) equal tde_eigvals."""
    import torch

    tde.set_defaults(fuse_few=32, wide_min=1 << 30)
    try:
        for fam, n in (("uniform", 65536), ("uniform", 9000)):
            d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_FAMILIES)
            dv, ev = _t(d), _t(e)
            _step(f"fuse_few=32 {fam} n={n}")
            lam_na = tde.eigvals_noalloc(dv, ev, leaf=64, leaf_dc=True, sweep_cols=8)
            torch.cuda.synchronize()
            lam_ref = tde.eigvals(dv, ev, leaf=64, leaf_dc=True, sweep_cols=8)
            assert np.array_equal(lam_na.cpu().numpy(), lam_ref.cpu().numpy())
            if n <= 9000:
                assert float(np.abs(lam_ref.cpu().numpy() - oracle.eigvals(d, e)).max()) <= GATE * tdgen.tnorm1(d, e)
    finally:
        tde.set_defaults()


def test_noalloc_status_and_limits(tde):
    import torch

    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    d, e = tdgen.tridiag("uniform", 3000)
    d = d.copy()
    d[1234] = np.nan
    _step("non-finite input")
    tde.eigvals_noalloc(_t(d), _t(e), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & 1  # the non-finite bit of the device status word
    # a clean call afterwards clears it
    d2, e2 = tdgen.tridiag("uniform", 3000)
    lam = tde.eigvals_noalloc(_t(d2), _t(e2), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert float(np.abs(lam.cpu().numpy() - oracle.eigvals(d2, e2)).max()) <= GATE * tdgen.tnorm1(d2, e2)
    _step("size beyond the scratch array")
    big = torch.zeros(65537, dtype=torch.float64, device="cuda:0")
    with pytest.raises(tde.TDEError) as ex:
        tde.eigvals_noalloc(big, big[:-1])
    assert ex.value.code == tde.TDE_EINVAL
    # n = 1 and n = 0
    one = tde.eigvals_noalloc(_t([3.5]), _t([]))
    assert float(one.item()) == 3.5
    assert tde.eigvals_noalloc(_t([]), _t([])).numel() == 0
