"""The host CPU boundary-row D&C baseline (libtde_host.so; the paper's CPU
design, Section 4.2) against the oracle: every eigenvalue within the gate on
every family, the Toeplitz closed form, reducible input through the driver's
split, the degenerate sizes, thread-count independence and argument errors.
No GPU."""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
import tdgen

GATE = 2e-11


@pytest.fixture(scope="module")
def hb():
    from paper_2605_26599_amd import build, host_br

    if not os.path.exists(host_br.LIB_PATH):
        build.build_host()
    host_br.lib()
    return host_br


@pytest.mark.parametrize("fam", ["uniform", "normal", "toeplitz", "wilkinson", "clustered", "paper_uniform",
                                 "paper_normal", "paper_toeplitz", "paper_clustered"])
@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 64, 65, 127, 1000, 2500])
def test_matches_oracle(hb, fam, n):
    d, e = tdgen.tridiag(fam, n)
    lam = hb.eigvals(d, e)
    ref = oracle.eigvals(d, e)
    assert np.all(np.diff(lam) >= 0)
    assert float(np.abs(lam - ref).max()) <= GATE * max(tdgen.tnorm1(d, e), 1e-300)


def test_toeplitz_closed_form(hb):
    n = 4096
    d, e = tdgen.tridiag("toeplitz", n)
    k = np.arange(1, n + 1, dtype=np.float64)
    ref = np.sort(2.0 - 2.0 * np.cos(k * math.pi / (n + 1)))
    assert float(np.abs(hb.eigvals(d, e) - ref).max()) <= 64 * np.finfo(float).eps * 4.0


def test_large_sampled(hb):
    n = 65536
    d, e = tdgen.tridiag("uniform", n, cfg=tdgen.CFG_FAMILIES)
    lam = hb.eigvals(d, e)
    ks = np.unique(np.concatenate([np.random.default_rng(3).choice(n, 256, replace=False), [0, n - 1]]))
    assert float(np.abs(lam[ks] - oracle.eigvals_index(d, e, ks)).max()) <= GATE * tdgen.tnorm1(d, e)
    # every eigenvalue, certified by two Sturm counts each
    assert oracle.certify(d, e, lam, GATE * tdgen.tnorm1(d, e)) == 0


def test_split_and_scale(hb):
    """Zero and negligible couplings split the matrix into blocks; blocks of
    wildly different magnitude are scaled on their own."""
    d, e = tdgen.tridiag("uniform", 3000)
    e = e.copy()
    e[::97] = 0.0
    e[500] = 1e-300
    d = d.copy()
    d[1000:1400] *= 2.0 ** 600
    e[1000:1399] *= 2.0 ** 600
    lam = hb.eigvals(d, e)
    ref = oracle.eigvals(d, e)
    assert float(np.abs(lam - ref).max()) <= GATE * tdgen.tnorm1(d, e)


def test_diagonal_and_constant(hb):
    d = np.random.default_rng(1).standard_normal(200)
    assert np.array_equal(hb.eigvals(d, np.zeros(199)), np.sort(d))
    lam = hb.eigvals(np.full(300, 3.0), np.full(299, 1e-9))
    assert float(np.abs(lam - oracle.eigvals(np.full(300, 3.0), np.full(299, 1e-9))).max()) <= GATE * 3.0


def test_thread_count_independent(hb):
    """Every merge runs the same arithmetic whichever thread takes it."""
    d, e = tdgen.tridiag("normal", 20000)
    a = hb.eigvals(d, e, threads=1)
    b = hb.eigvals(d, e, threads=4)
    assert np.array_equal(a, b)


def test_workspace_and_errors(hb):
    assert hb.workspace(1000) == (16000, 2000)
    L = hb.lib()
    dp = ctypes.POINTER(ctypes.c_double)
    d2, e2, lam = np.array([1.0, 2.0]), np.array([0.5]), np.zeros(2)
    work = np.zeros(32, dtype=np.float64)
    iw = np.zeros(4, dtype=np.int32)
    ip = iw.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    args = (d2.ctypes.data_as(dp), e2.ctypes.data_as(dp))
    lp, wp = lam.ctypes.data_as(dp), work.ctypes.data_as(dp)
    assert L.tde_host_eigvals(*args, -1, lp, wp, 32, ip, 4, 0) == hb.TDE_HOST_EINVAL
    assert L.tde_host_eigvals(*args, 2, lp, wp, 32, ip, 3, 0) == hb.TDE_HOST_EINVAL  # iwork too small
    assert L.tde_host_eigvals(*args, 2, lp, wp, 31, ip, 4, 0) == hb.TDE_HOST_EINVAL  # needs 16 n doubles
    assert L.tde_host_eigvals(*args, 2, lp, wp, 32, ip, 4, -1) == hb.TDE_HOST_EINVAL
    assert L.tde_host_eigvals(*args, 0, lp, wp, 0, ip, 0, 0) == hb.TDE_HOST_OK
    assert L.tde_host_eigvals(*args, 2, lp, wp, 32, ip, 4, 0) == hb.TDE_HOST_OK
    assert np.allclose(lam, [1.5 - math.hypot(0.5, 0.5), 1.5 + math.hypot(0.5, 0.5)], rtol=0, atol=4e-16)
    d = np.array([1.0, np.nan])
    with pytest.raises(RuntimeError):
        hb.eigvals(d, np.array([0.5]))
