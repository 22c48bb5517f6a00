"""Failure handling and cache management of the HIP path, forced from the host.

* Non-convergence: a secular iteration cap of one sweep per root (the
  max_sweeps option) makes roots stop unconverged, and every kernel path that
  solves roots (level-wide, fused small merges, whole-merge workgroups,
  in-wave levels, wide sweeps, in-wave leaves) must report TDE_ENOCONV while
  still exiting normally.
* Graph cache: more distinct buffer sets than the cache holds, replayed
  without synchronising in between, must each give the eager result bit for
  bit (an executable still queued must never be destroyed).
* Plan cache: many distinct problem shapes leave a bounded number of plans.
"""
import numpy as np
import pytest

import oracle
import tdgen

pytestmark = pytest.mark.gpu

GATE = 2e-11


def _step(msg):
    print(f"[gpu-robust] {msg}", flush=True)


@pytest.fixture(scope="module")
def tde():
    import torch

    import paper_2605_26599_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def _dev():
    import torch

    return torch.device("cuda:0")


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(_dev())


@pytest.mark.parametrize("kw", [{}, {"leaf": 4}, {"leaf": 64, "leaf_dc": True}, {"wide_min": 2},
                                {"leaf": 64, "leaf_dc": True, "wide_min": 32, "sweep_cols": 64}])
def test_forced_nonconvergence(tde, kw):
    d, e = tdgen.tridiag("uniform", 6000)
    dv, ev = _t(d), _t(e)
    try:
        tde.set_defaults(max_sweeps=1)
        _step(f"max_sweeps=1 {kw}")
        with pytest.raises(tde.TDEError) as ex:
            tde.eigvals(dv, ev, **kw)
        assert ex.value.code == tde.TDE_ENOCONV
    finally:
        tde.set_defaults()
    _step(f"default cap {kw}")
    lam = tde.eigvals(dv, ev, **kw).cpu().numpy()
    assert np.abs(lam - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e)


def test_forced_nonconvergence_waved_levels_and_tiles(tde):
    """The in-wave levels (1500 problems of 40..64 columns at leaf 8: every
    level of many small merges runs in waves) and the regular tiles that take
    the few-merge levels' larger merges under fuse_few report the cap and
    non-finite input like every other path."""
    probs = [tdgen.tridiag("uniform", 40 + (i % 25), inst=i) for i in range(1500)]
    bt = tdgen.pack(probs)
    bd, be = _t(bt.d), _t(bt.e)
    d, e = tdgen.tridiag("uniform", 9000)
    dv, ev = _t(d), _t(e)
    try:
        tde.set_defaults(max_sweeps=1)
        _step("max_sweeps=1 waved batch")
        with pytest.raises(tde.TDEError) as ex:
            tde.eigvals_batched(bd, be, bt.offsets, leaf=8)
        assert ex.value.code == tde.TDE_ENOCONV
        _step("max_sweeps=1 fuse_few 32 regular tiles")
        with pytest.raises(tde.TDEError) as ex:
            tde.eigvals(dv, ev, leaf=64, leaf_dc=True, fuse_few=32, wide_min=1 << 30)
        assert ex.value.code == tde.TDE_ENOCONV
    finally:
        tde.set_defaults()
    _step("non-finite entry in a waved batch")
    bad = bt.d.copy()
    bad[int(bt.offsets[700]) + 3] = np.inf
    with pytest.raises(tde.TDEError) as ex:
        tde.eigvals_batched(_t(bad), be, bt.offsets, leaf=8)
    assert ex.value.code == tde.TDE_ENONFINITE
    _step("default cap waved batch")
    lam = tde.eigvals_batched(bd, be, bt.offsets, leaf=8).cpu().numpy()
    for b in range(0, bt.count, 149):
        db, eb = bt.problem(b)
        lo, hi = int(bt.offsets[b]), int(bt.offsets[b + 1])
        assert np.abs(lam[lo:hi] - oracle.eigvals(db, eb)).max() <= GATE * tdgen.tnorm1(db, eb)


def test_forced_nonconvergence_reverse_mode(tde):
    d, e = tdgen.tridiag("uniform", 3000, cfg=tdgen.CFG_GRAD)
    try:
        tde.set_defaults(max_sweeps=1)
        _step("max_sweeps=1 checkpointing forward")
        with pytest.raises(tde.TDEError) as ex:
            tde.eigvals_ckpt(_t(d), _t(e))
        assert ex.value.code == tde.TDE_ENOCONV
    finally:
        tde.set_defaults()


def test_graph_cache_eviction_while_queued(tde):
    """80 distinct output buffers (more than the 64 cached graphs): every solve
    is a new capture that evicts an older executable while earlier replays may
    still be queued; no synchronisation until the end."""
    import torch

    n = 3000
    d, e = tdgen.tridiag("uniform", n)
    dv, ev = _t(d), _t(e)
    ref = tde.eigvals(dv, ev, graph=False).cpu().numpy()
    outs = [torch.empty(n, dtype=torch.float64, device=_dev()) for _ in range(80)]
    _step("80 captures without sync")
    for rnd in range(2):
        for o in outs:
            tde.eigvals(dv, ev, out=o, check=False)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref), i
    sizes = tde.cache_sizes()
    assert sizes["graphs"] <= 64, sizes


def test_plan_cache_bounded(tde):
    import torch

    _step("40 distinct sizes")
    results = []
    for i in range(40):
        n = 500 + 37 * i
        d, e = tdgen.tridiag("normal", n, inst=i)
        lam = tde.eigvals(_t(d), _t(e), check=False)
        results.append((d, e, lam))
    torch.cuda.synchronize()
    assert tde.cache_sizes()["plans"] <= 32
    for d, e, lam in results:
        assert np.abs(lam.cpu().numpy() - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e)
    _step("release plans")
    tde.release_plans()
    assert tde.cache_sizes() == {"plans": 0, "graphs": 0, "split_schedules": 0}
    d, e = tdgen.tridiag("uniform", 777)
    lam = tde.eigvals(_t(d), _t(e)).cpu().numpy()
    assert np.abs(lam - oracle.eigvals(d, e)).max() <= GATE * tdgen.tnorm1(d, e)
