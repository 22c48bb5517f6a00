"""Reverse mode of the HIP path (through the C-ABI) against the dense
Hellmann-Feynman gradient of the oracle.

Loss L = sum_k w_k lambda_k.  Gates (per problem, normwise):
  ||g_d - g_d^HF||_inf / ||g_d^HF||_inf <= 1e-7, and the same for e;
  invariants sum_i g_d,i = sum_k w_k and d . g_d + e . g_e = L to 1e-12
  relative; on sampled coordinates |g_i - FD_i| <= |g_i^HF - FD_i| + 1e-7 ||g^HF||,
  with FD the central difference (h = 1e-6) of the bisection oracle.
Gradients of nearly multiple eigenvalues are ill-conditioned for uneven
weights (Wilkinson pairs agree to far below 1e-16 relative at n >= 21), so the
Wilkinson family uses weights that are a smooth function of lambda.
"""
import numpy as np
import pytest

import oracle
import tdgen

pytestmark = pytest.mark.gpu

GATE = 1e-7


def _step(msg):
    print(f"[gpu-grad] {msg}", flush=True)


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

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(_dev())


def _weights(fam, d, e, n):
    if fam == "wilkinson":
        return np.cos(0.37 * oracle.eigvals(d, e))
    return tdgen.loss_weights(n)


def _grad_single(tde, d, e, w, leaf=None, graph=True):
    n = len(d)
    dv, ev = _t(d), _t(e if len(e) else np.zeros(1))
    lam, ck = tde.eigvals_ckpt(dv, ev, leaf=leaf, graph=graph)
    gd, ge = tde.eigvals_backward(dv, ev, _t(w), ck, leaf=leaf, graph=graph)
    return lam.cpu().numpy(), gd.cpu().numpy(), ge.cpu().numpy()[: max(n - 1, 0)]


def _rel(a, b):
    s = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / s) if b.size and s > 0 else float(np.abs(a - b).max() if a.size else 0.0)


def _check_hf(d, e, w, lam, gd, ge):
    lr, gdr, ger = oracle.grad_reference(d, e, w)
    assert np.abs(lam - lr).max() <= 2e-11 * tdgen.tnorm1(d, e)
    ed, ee = _rel(gd, gdr), _rel(ge, ger)
    assert ed <= GATE and ee <= GATE, (ed, ee)
    return ed, ee, gdr, ger


def _check_invariants(d, e, w, lam, gd, ge):
    L = float(np.dot(w, lam))
    sw = np.abs(w).sum()
    assert abs(gd.sum() - w.sum()) <= 1e-12 * sw
    assert abs(np.dot(d, gd) + np.dot(e, ge) - L) <= 1e-12 * sw * tdgen.tnorm1(d, e)


# --- every family, ragged sizes, several leaf sizes ---------------------------

@pytest.mark.parametrize("fam", ["uniform", "normal", "toeplitz", "wilkinson", "clustered"])
@pytest.mark.parametrize("leaf", [1, 4, 8, 32])
def test_grad_families(tde, fam, leaf):
    for n in [1, 2, 3, 5, 33, 100, 257, 1000]:
        _step(f"fam={fam} leaf={leaf} n={n}")
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_GRAD)
        w = _weights(fam, d, e, n)
        lam, gd, ge = _grad_single(tde, d, e, w, leaf=leaf)
        _check_hf(d, e, w, lam, gd, ge)
        _check_invariants(d, e, w, lam, gd, ge)


def test_grad_edge_cases(tde):
    _step("n=1")
    lam, gd, ge = _grad_single(tde, np.array([0.7]), np.zeros(0), np.array([-1.5]))
    assert lam[0] == 0.7 and gd[0] == -1.5 and ge.size == 0
    _step("n=2 closed form")
    a, b, c = 0.3, -1.1, 0.45
    w = np.array([0.8, -0.25])
    lam, gd, ge = _grad_single(tde, np.array([a, b]), np.array([c]), w)
    r = np.hypot((a - b) / 2, c)
    # lambda_+- = (a+b)/2 +- r; dr/da = (a-b)/(4r), dr/db = -(a-b)/(4r), dr/dc = c/r
    dra, drb, drc = (a - b) / (4 * r), -(a - b) / (4 * r), c / r
    ref_d = np.array([w.sum() / 2 + (w[1] - w[0]) * dra, w.sum() / 2 + (w[1] - w[0]) * drb])
    ref_e = np.array([(w[1] - w[0]) * drc])
    assert np.abs(gd - ref_d).max() <= 1e-14 and np.abs(ge - ref_e).max() <= 1e-14
    _step("decoupled (e = 0): g_d = w permuted onto sorted d, g_e = 0")
    d, _ = tdgen.tridiag("normal", 300, cfg=tdgen.CFG_GRAD)
    w = tdgen.loss_weights(300)
    lam, gd, ge = _grad_single(tde, d, np.zeros(299), w)
    ref = np.empty(300)
    ref[np.argsort(d, kind="stable")] = w
    assert np.array_equal(gd, ref) and np.all(ge == 0.0)
    _step("scaled input: gradient is scale invariant")
    d, e = tdgen.tridiag("uniform", 700, cfg=tdgen.CFG_GRAD)
    w = tdgen.loss_weights(700)
    _, gd1, ge1 = _grad_single(tde, d, e, w)
    _, gd2, ge2 = _grad_single(tde, d * 2.0**40, e * 2.0**40, w)
    assert _rel(gd2, gd1) <= 1e-13 and _rel(ge2, ge1) <= 1e-13


# --- C5 (i): n = 8192 --------------------------------------------------------

def test_c5_single_8192(tde):
    n = 8192
    _step("C5 single n=8192")
    d, e = tdgen.tridiag("uniform", n, cfg=tdgen.CFG_GRAD)
    w = tdgen.loss_weights(n)
    lam, gd, ge = _grad_single(tde, d, e, w)
    ed, ee, gdr, ger = _check_hf(d, e, w, lam, gd, ge)
    _check_invariants(d, e, w, lam, gd, ge)
    print(f"C5 n=8192 rel err d {ed:.2e} e {ee:.2e}")
    # coordinate-wise central differences of the oracle on a few coordinates
    h = 1e-6
    gmax = max(np.abs(gdr).max(), np.abs(ger).max())
    for kind, i in [("d", 0), ("d", 4097), ("e", 1), ("e", 8190)]:
        _step(f"C5 FD {kind}[{i}]")
        dp, dm, ep, em = d.copy(), d.copy(), e.copy(), e.copy()
        if kind == "d":
            dp[i] += h
            dm[i] -= h
            mine, ref = gd[i], gdr[i]
        else:
            ep[i] += h
            em[i] -= h
            mine, ref = ge[i], ger[i]
        fd = (np.dot(w, oracle.eigvals(dp, ep)) - np.dot(w, oracle.eigvals(dm, em))) / (2 * h)
        assert abs(mine - fd) <= abs(ref - fd) + GATE * gmax


# --- C5 (ii): 256 x n = 1024 -------------------------------------------------

def test_c5_batched_256x1024(tde):
    _step("C5 batched 256 x 1024")
    probs = [tdgen.tridiag("uniform", 1024, cfg=tdgen.CFG_GRAD, inst=b) for b in range(256)]
    bt = tdgen.pack(probs)
    ws = [tdgen.loss_weights(1024, inst=b) for b in range(256)]
    offs = [int(x) for x in bt.offsets]
    dv, ev = _t(bt.d), _t(bt.e)
    lam, ck = tde.eigvals_ckpt(dv, ev, offsets=offs)
    gd, ge = tde.eigvals_backward(dv, ev, _t(np.concatenate(ws)), ck, offsets=offs)
    lam, gd, ge = lam.cpu().numpy(), gd.cpu().numpy(), ge.cpu().numpy()
    worst = 0.0
    for b in range(256):
        s, t = offs[b], offs[b + 1]
        d, e = probs[b]
        assert ge[t - 1] == 0.0
        _check_invariants(d, e, ws[b], lam[s:t], gd[s:t], ge[s:t - 1])
        ed, ee, _, _ = _check_hf(d, e, ws[b], lam[s:t], gd[s:t], ge[s:t - 1])
        worst = max(worst, ed, ee)
    print(f"C5 batched worst rel err {worst:.2e}")


def test_batched_grad_matches_single(tde):
    """Mixed sizes (including 0 and 1) in one batch give the same gradients,
    bit for bit, as each problem solved alone with the same leaf."""
    sizes = [0, 1, 2, 17, 300, 0, 64, 1025, 5]
    probs = [tdgen.tridiag("normal", s, cfg=tdgen.CFG_GRAD, inst=i) for i, s in enumerate(sizes)]
    bt = tdgen.pack(probs)
    ws = [tdgen.loss_weights(s, inst=i) for i, s in enumerate(sizes)]
    offs = [int(x) for x in bt.offsets]
    dv, ev = _t(bt.d), _t(bt.e if len(bt.e) else np.zeros(1))
    lam, ck = tde.eigvals_ckpt(dv, ev, offsets=offs, leaf=8)
    gd, ge = tde.eigvals_backward(dv, ev, _t(np.concatenate(ws)), ck, offsets=offs, leaf=8)
    gd, ge = gd.cpu().numpy(), ge.cpu().numpy()
    for b, (d, e) in enumerate(probs):
        s, t = offs[b], offs[b + 1]
        if t == s:
            continue
        _, gd1, ge1 = _grad_single(tde, d, e, ws[b], leaf=8)
        assert np.array_equal(gd[s:t], gd1)
        assert np.array_equal(ge[s:t - 1], ge1) and ge[t - 1] == 0.0


# --- autograd, graphs, determinism --------------------------------------------

def test_autograd_function(tde):
    import torch

    for offsets in [None, "batch"]:
        _step(f"autograd offsets={offsets}")
        if offsets is None:
            d, e = tdgen.tridiag("uniform", 3000, cfg=tdgen.CFG_GRAD)
            offs = None
            w = tdgen.loss_weights(3000)
        else:
            probs = [tdgen.tridiag("uniform", s, cfg=tdgen.CFG_GRAD, inst=i) for i, s in enumerate([100, 1, 777])]
            bt = tdgen.pack(probs)
            d, e, offs = bt.d, bt.e, [int(x) for x in bt.offsets]
            w = np.concatenate([tdgen.loss_weights(s, inst=i) for i, s in enumerate([100, 1, 777])])
        dv = _t(d).requires_grad_(True)
        ev = _t(e).requires_grad_(True)
        lam = tde.differentiable_eigvals(dv, ev, offsets=offs)
        (lam * _t(w)).sum().backward()
        lam2, ck = tde.eigvals_ckpt(_t(d), _t(e), offsets=offs)
        gd, ge = tde.eigvals_backward(_t(d), _t(e), _t(w), ck, offsets=offs)
        assert torch.equal(lam.detach(), lam2)
        assert torch.equal(dv.grad, gd)
        m = ev.numel()
        assert torch.equal(ev.grad[: min(m, ge.numel())], ge[: min(m, ge.numel())])


def test_backward_graph_replays_match_eager(tde):
    """Captured forward-with-checkpoint and backward graphs, replayed several
    times with unrelated eager work in between, match the eager passes bitwise."""
    import torch

    for fam, n, leaf in [("uniform", 5000, None), ("toeplitz", 3001, 4), ("clustered", 4096, 32)]:
        _step(f"graph vs eager fam={fam} n={n} leaf={leaf}")
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_GRAD)
        w = _t(tdgen.loss_weights(n))
        dv, ev = _t(d), _t(e)
        lam0, ck0 = tde.eigvals_ckpt(dv, ev, leaf=leaf, graph=False)
        gd0, ge0 = tde.eigvals_backward(dv, ev, w, ck0, leaf=leaf, graph=False)
        out = torch.empty(n, dtype=torch.float64, device=_dev())
        ck = torch.empty_like(ck0)
        for rep in range(3):
            lam, _ = tde.eigvals_ckpt(dv, ev, leaf=leaf, out=out, ckpt=ck, graph=True)
            gd, ge = tde.eigvals_backward(dv, ev, w, ck, leaf=leaf, graph=True)
            torch.cuda.synchronize()
            assert torch.equal(lam, lam0) and torch.equal(gd, gd0) and torch.equal(ge, ge0), (fam, rep)
            junk = tde.eigvals(dv[: n // 3].contiguous(), ev[: n // 3 - 1].contiguous(), graph=False)
            torch.cuda.synchronize()
            assert junk.numel() == n // 3


def test_grad_through_wide_sweep(tde):
    """Roots found by the wide secular sweep feed the same reverse pass."""
    for fam, n in [("uniform", 3000), ("toeplitz", 2000), ("clustered", 1500)]:
        _step(f"wide_min=2 fam={fam} n={n}")
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_GRAD)
        w = tdgen.loss_weights(n)
        dv, ev = _t(d), _t(e)
        lam, ck = tde.eigvals_ckpt(dv, ev, wide_min=2)
        gd, ge = tde.eigvals_backward(dv, ev, _t(w), ck, wide_min=2)
        _check_hf(d, e, w, lam.cpu().numpy(), gd.cpu().numpy(), ge.cpu().numpy()[: n - 1])


def test_backward_lanes_per_root_variants(tde):
    for cols in [1, 4, 64]:
        for fam, n in [("uniform", 4000), ("toeplitz", 2000)]:
            _step(f"sweep_cols={cols} fam={fam} n={n}")
            d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_GRAD)
            w = tdgen.loss_weights(n)
            dv, ev = _t(d), _t(e)
            lam, ck = tde.eigvals_ckpt(dv, ev, sweep_cols=cols)
            gd, ge = tde.eigvals_backward(dv, ev, _t(w), ck, sweep_cols=cols)
            _check_hf(d, e, w, lam.cpu().numpy(), gd.cpu().numpy(), ge.cpu().numpy()[: n - 1])


@pytest.mark.parametrize("wide_min", [None, 1 << 30])
def test_grad_with_fuse_few(tde, wide_min):
    """Roots of the few-merge levels' larger merges taken by the root-parallel
    kernels (fuse_few 32; the regular tiles when wide_min is 2^30) feed the
    same reverse pass, single and batched."""
    for fam, n in [("uniform", 8192), ("toeplitz", 2000), ("clustered", 3000)]:
        _step(f"fuse_few=32 wide_min={wide_min} fam={fam} n={n}")
        d, e = tdgen.tridiag(fam, n, cfg=tdgen.CFG_GRAD)
        w = tdgen.loss_weights(n)
        dv, ev = _t(d), _t(e)
        lam, ck = tde.eigvals_ckpt(dv, ev, leaf=8, fuse_few=32, wide_min=wide_min)
        gd, ge = tde.eigvals_backward(dv, ev, _t(w), ck, leaf=8, fuse_few=32, wide_min=wide_min)
        _check_hf(d, e, w, lam.cpu().numpy(), gd.cpu().numpy(), ge.cpu().numpy()[: n - 1])
    _step(f"fuse_few=32 wide_min={wide_min} batched")
    probs = [tdgen.tridiag("uniform", s, cfg=tdgen.CFG_GRAD, inst=i) for i, s in enumerate([1500, 40, 900, 2049])]
    bt = tdgen.pack(probs)
    w = tdgen.loss_weights(int(bt.offsets[-1]))
    dv, ev = _t(bt.d), _t(bt.e)
    lam, ck = tde.eigvals_ckpt(dv, ev, bt.offsets, leaf=8, fuse_few=32, wide_min=wide_min)
    gd, ge = tde.eigvals_backward(dv, ev, _t(w), ck, bt.offsets, leaf=8, fuse_few=32, wide_min=wide_min)
    lam, gd, ge = lam.cpu().numpy(), gd.cpu().numpy(), ge.cpu().numpy()
    for b, (db, eb) in enumerate(probs):
        lo, hi = int(bt.offsets[b]), int(bt.offsets[b + 1])
        _check_hf(db, eb, w[lo:hi], lam[lo:hi], gd[lo:hi], ge[lo:hi - 1])
