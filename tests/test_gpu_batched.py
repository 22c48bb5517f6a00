"""Batched API parity: many packed tridiagonals of uneven size merged level by
level in shared launches, checked problem by problem against the oracle."""
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

    assert torch.cuda.is_available()
    m.lib()
    return m


def _solve_batch(tde, batch, leaf=None):
    import torch

    dev = torch.device("cuda:0")
    d = torch.from_numpy(batch.d).to(dev)
    e = torch.from_numpy(batch.e).to(dev)
    return tde.eigvals_batched(d, e, batch.offsets, leaf=leaf).cpu().numpy()


def _check_problem(batch, lam, b, full=True):
    d, e = batch.problem(b)
    lo, hi = int(batch.offsets[b]), int(batch.offsets[b + 1])
    got = lam[lo:hi]
    if hi == lo:
        return
    tn = tdgen.tnorm1(d, e)
    assert np.all(np.diff(got) >= 0)
    if full:
        ref = oracle.eigvals(d, e)
        assert np.abs(got - ref).max() <= GATE * tn, b
    else:
        assert oracle.certify(d, e, got, GATE * tn) == 0, b


@pytest.mark.parametrize("leaf", [1, 4, 32])
def test_mixed_sizes_small(tde, leaf):
    _step(f"mixed sizes leaf={leaf}")
    g = np.random.default_rng(5)
    sizes = [0, 1, 2, 3, 0, 17, 32, 33, 64, 65, 1, 500, 1023, 7, 0]
    fams = ["uniform", "toeplitz", "wilkinson", "clustered", "normal"]
    probs = [tdgen.tridiag(fams[i % len(fams)], s, inst=i) for i, s in enumerate(sizes)]
    probs += [tdgen.tridiag("uniform", int(s), inst=100 + i) for i, s in enumerate(g.integers(1, 300, 40))]
    batch = tdgen.pack(probs)
    lam = _solve_batch(tde, batch, leaf)
    for b in range(batch.count):
        _check_problem(batch, lam, b)


def test_batched_equals_single(tde):
    import torch

    _step("batched == single, bitwise")
    batch = tdgen.batched("uniform", count=64, lo=32, hi=2048, inst=3)
    lam = _solve_batch(tde, batch)
    dev = torch.device("cuda:0")
    for b in range(0, batch.count, 7):
        d, e = batch.problem(b)
        one = tde.eigvals(torch.from_numpy(d.copy()).to(dev), torch.from_numpy(e.copy()).to(dev)).cpu().numpy()
        lo, hi = int(batch.offsets[b]), int(batch.offsets[b + 1])
        assert np.array_equal(one, lam[lo:hi]), b


@pytest.mark.parametrize("fam", ["uniform", "clustered", "wilkinson"])
def test_wave_levels_equal_block_levels(tde, fam):
    """Levels of more than 1024 merges of at most 64 columns run one wave per
    pack of merges, levels of fewer merges one workgroup per merge; the roots
    take the same canonical sums either way, so a problem's eigenvalues do not
    depend on how many problems share its levels (1500 problems of 40..64
    columns at leaf 8: every level waved, root merges included; their first 64
    alone: every level in workgroups)."""
    _step(f"in-wave levels == whole-merge workgroups, {fam}")
    probs = [tdgen.tridiag(fam, 40 + (i % 25), inst=i) for i in range(1500)]
    big, small = tdgen.pack(probs), tdgen.pack(probs[:64])
    a = _solve_batch(tde, big, leaf=8)
    b = _solve_batch(tde, small, leaf=8)
    n = int(small.offsets[-1])
    assert np.array_equal(a[:n], b)
    for p in range(0, 64, 9):
        _check_problem(small, b, p)
    for p in range(64, 1500, 97):
        _check_problem(big, a, p)


def test_c4_batched_4096(tde):
    """Every problem of the batch: 48 bisected in full, all 4096 certified
    eigenvalue by eigenvalue with two Sturm counts each."""
    _step("C4: 4096 problems, log-uniform sizes in [32, 4096]")
    batch = tdgen.batched("uniform", count=4096, lo=32, hi=4096, inst=0)
    lam = _solve_batch(tde, batch)
    g = np.random.default_rng(11)
    full = set(g.choice(batch.count, 48, replace=False).tolist())
    for b in range(batch.count):
        _check_problem(batch, lam, b, full=b in full)
        if b in full:
            _check_problem(batch, lam, b, full=False)


@pytest.mark.parametrize("fam", ["uniform", "toeplitz", "clustered"])
def test_group_max_does_not_change_results(tde, fam):
    """The fused small merges sum in one fixed tree whatever the lanes per
    root: every group_max gives the same bits, single and batched."""
    import torch

    dev = torch.device("cuda:0")
    d, e = tdgen.tridiag(fam, 9000)
    dv, ev = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
    tol = GATE * tdgen.tnorm1(d, e)
    exact = oracle.eigvals(d, e)
    for kw in ({}, {"leaf": 64, "leaf_dc": True}, {"leaf": 16}):
        ref = None
        for gm in (None, 4, 8, 16):
            _step(f"group_max={gm} {fam} {kw}")
            lam = tde.eigvals(dv, ev, group_max=gm, **kw).cpu().numpy()
            if ref is None:
                ref = lam
                assert np.abs(lam - exact).max() <= tol
            else:
                assert np.array_equal(lam, ref), (gm, kw)
    batch = tdgen.batched(fam if fam != "toeplitz" else "uniform", count=300, lo=32, hi=1500, inst=5)
    bd, be = torch.from_numpy(batch.d).to(dev), torch.from_numpy(batch.e).to(dev)
    outs = [tde.eigvals_batched(bd, be, batch.offsets, group_max=gm).cpu().numpy() for gm in (None, 4, 8, 16)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
