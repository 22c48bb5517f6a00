"""Leaves solved by divide and conquer inside one wave (TDE_FLAG_LEAF_DC).

The in-wave leaf runs the leaf's own merge tree down to single columns, so a
plan with leaf bound L and DC leaves performs the same merges as a plan with
leaf bound 1 (the global levels below L move into the leaf kernel).  Checks:
the eigenvalue gate against the oracle on every family, ragged leaf sizes and
whole problems that fit in one leaf; agreement with the leaf-1 global path to
a few ulps of ||T||; boundary rows; batched layouts; work counters.
"""
import numpy as np
import pytest

import oracle
import tdgen

pytestmark = pytest.mark.gpu

GATE = 2e-11


def _step(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def tde():
    import torch

    import paper_2605_26599_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _dev():
    import torch

    return torch.device("cuda:0")


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x if len(x) else np.zeros(1))).to(_dev())


def _dc(tde, d, e, leaf, **kw):
    return tde.eigvals(_t(d), _t(e), leaf=leaf, leaf_dc=True, **kw).cpu().numpy()


@pytest.mark.parametrize("fam", ["uniform", "normal", "toeplitz", "wilkinson", "clustered",
                                 "paper_uniform", "paper_toeplitz", "paper_clustered"])
@pytest.mark.parametrize("leaf", [2, 5, 16, 33, 64])
def test_families(tde, fam, leaf):
    for n in [1, 2, 3, 4, 7, 31, 32, 33, 63, 64, 65, 127, 200, 1000, 2049]:
        _step(f"dc fam={fam} leaf={leaf} n={n}")
        d, e = tdgen.tridiag(fam, n)
        lam = _dc(tde, d, e, leaf)
        assert np.all(np.diff(lam) >= 0), "output not ascending"
        err = np.abs(lam - oracle.eigvals(d, e)).max()
        assert err <= GATE * tdgen.tnorm1(d, e), (fam, leaf, n, err)


@pytest.mark.parametrize("n", [64, 1000, 4096, 65536])
@pytest.mark.parametrize("fam", ["uniform", "toeplitz", "clustered"])
def test_matches_leaf1_global_path(tde, fam, n):
    """Same merges, same per-merge arithmetic: the DC leaf-64 result equals the
    all-global leaf-1 result to a few ulps of ||T|| (bitwise in practice)."""
    _step(f"dc vs leaf1 fam={fam} n={n}")
    d, e = tdgen.tridiag(fam, n)
    a = _dc(tde, d, e, 64, sweep_cols=64)
    b = tde.eigvals(_t(d), _t(e), leaf=1, sweep_cols=64, wide_min=1 << 30).cpu().numpy()
    tn = tdgen.tnorm1(d, e)
    diff = np.abs(a - b).max()
    print(f"dc vs leaf1: max diff {diff:.3e} = {diff / tn / np.finfo(float).eps:.2f} eps ||T||")
    assert diff <= 16 * np.finfo(float).eps * tn


def test_edge_cases(tde):
    _step("dc edge: zero matrix")
    assert np.all(_dc(tde, np.zeros(300), np.zeros(299), 64) == 0.0)
    _step("dc edge: diagonal")
    d, _ = tdgen.tridiag("normal", 777)
    assert np.array_equal(_dc(tde, d, np.zeros(776), 64), np.sort(d))
    _step("dc edge: zeros in e")
    d, e = tdgen.tridiag("uniform", 1500)
    e[::7] = 0.0
    assert np.abs(_dc(tde, d, e, 64) - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e)
    _step("dc edge: duplicate blocks and constant diagonal")
    d1, e1 = tdgen.tridiag("uniform", 16)
    d = np.tile(d1, 64)
    e = np.concatenate([np.concatenate([e1, [1e-3]]) for _ in range(64)])[:-1]
    assert np.abs(_dc(tde, d, e, 64) - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e)
    d, e = np.ones(1000), np.full(999, 1e-14)
    assert np.abs(_dc(tde, d, e, 32) - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e)
    _step("dc edge: scales")
    d, e = tdgen.tridiag("uniform", 900)
    for s in [2.0**600, 2.0**-600, 1e300, 3e-300]:
        lam = _dc(tde, d * s, e * s, 64)
        assert np.abs(lam - oracle.eigvals(d * s, e * s)).max() <= GATE * tdgen.tnorm1(d * s, e * s)


def test_nonfinite(tde):
    d, e = tdgen.tridiag("uniform", 500)
    d[100] = np.nan
    with pytest.raises(tde.TDEError) as ex:
        _dc(tde, d, e, 64)
    assert ex.value.code == tde.TDE_ENONFINITE


def test_batched_ragged(tde):
    _step("dc batched ragged")
    sizes = [0, 1, 2, 3, 64, 65, 17, 500, 1025, 31, 4096]
    probs = [tdgen.tridiag("uniform" if i % 2 else "toeplitz", s, inst=i) for i, s in enumerate(sizes)]
    bt = tdgen.pack(probs)
    for leaf in [8, 64]:
        lam = tde.eigvals_batched(_t(bt.d), _t(bt.e), bt.offsets, leaf=leaf, leaf_dc=True).cpu().numpy()
        for b, (d, e) in enumerate(probs):
            s, t = int(bt.offsets[b]), int(bt.offsets[b + 1])
            if t > s:
                assert np.abs(lam[s:t] - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e), (leaf, b)


def test_rows(tde):
    """Boundary rows through DC leaves (including whole problems inside one
    leaf) against the oracle's eigenvectors, away from close eigenvalues."""
    for n in [1, 2, 5, 40, 64, 300]:
        _step(f"dc rows n={n}")
        d, e = tdgen.tridiag("normal", n, inst=3)
        lam, q0, q1 = tde.eigvals_rows(_t(d), _t(e), leaf=64, leaf_dc=True)
        lam, q0, q1 = lam.cpu().numpy(), q0.cpu().numpy(), q1.cpu().numpy()
        rl, r0, r1 = oracle.boundary_rows(d, e)
        tn = tdgen.tnorm1(d, e)
        assert np.abs(lam - rl).max() <= GATE * tn
        gap = np.full(n, np.inf)
        if n > 1:
            g = np.diff(rl)
            gap[:-1] = g
            gap[1:] = np.minimum(gap[1:], g)
        tol = 1e-10 + 64 * np.finfo(float).eps * tn / gap
        assert np.all(np.abs(np.abs(q0) - np.abs(r0)) <= tol)
        assert np.all(np.abs(np.abs(q1) - np.abs(r1)) <= tol)
        assert np.all(np.abs(q0 * q1 - r0 * r1) <= 2 * tol)


def test_counters(tde):
    import torch

    d, e = tdgen.tridiag("uniform", 4096)
    ws = torch.empty(tde.workspace_bytes(4096, 1, 64), dtype=torch.uint8, device=_dev())
    tde.eigvals(_t(d), _t(e), leaf=64, leaf_dc=True, workspace=ws)
    torch.cuda.synchronize()
    c = tde.counters(ws)
    assert c["leaf_columns"] == 4096
    assert c["leaf_rotations"] == 0
    # every level of the leaf-1 tree: log2(4096) = 12 levels of 4096 columns
    assert c["merge_columns"] == 12 * 4096
    # six levels inside the 64-column leaves, six global ones: both did work
    assert c["dc_roots"] > 0 and c["roots"] > 0
    assert c["dc_secular_terms"] >= c["dc_roots"]
    # the global levels' roots: whole-merge workgroups (merges of at most 512
    # columns) plus the fused root kernel make up all of them here
    assert c["level_roots"] > 0
    assert c["level_roots"] + c["small_roots"] == c["roots"]
    assert c["level_secular_terms"] + c["small_secular_terms"] == c["secular_terms"]
    # the global path alone counts no in-wave work
    tde.eigvals(_t(d), _t(e), leaf=64, leaf_dc=False, workspace=ws)
    torch.cuda.synchronize()
    c = tde.counters(ws)
    assert c["dc_roots"] == 0 and c["dc_secular_terms"] == 0 and c["leaf_rotations"] > 0
