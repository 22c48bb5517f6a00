"""The library's host planning code and the leaf eigensolver's arithmetic,
built for the CPU with g++ under AddressSanitizer and UBSan (no GPU needed).

tests/host/host_check.cpp compiles tde_planner.cpp (merge-tree tables,
block-to-merge maps, workspace / checkpoint / reverse-pass carving) and the
device header's leaf QL as plain host C++.  The plan mode checks the tables
and carvings of 400 random batches; the leaf mode returns eigenvalues and the
first and last eigenvector rows of one leaf, compared here with LAPACK; the
search mode checks the assembly's partition-point searches.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import tdgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "host", "host_check.cpp"),
       os.path.join(ROOT, "paper_2605_26599_amd", "csrc", "tde_planner.cpp")]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("host") / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", "-o", out] + SRC
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    return env


def test_plan_tables_and_carving(exe):
    r = subprocess.run([exe, "plan"], capture_output=True, text=True, env=_env(), timeout=600)
    assert r.returncode == 0 and "plan ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


def test_assembly_searches(exe):
    """The assembly's partition-point searches, binary and 8-way, equal a
    linear count on ascending lists with repeats (lengths 0 to 70000)."""
    r = subprocess.run([exe, "search"], capture_output=True, text=True, env=_env(), timeout=600)
    assert r.returncode == 0 and "search ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


def _leaf(exe, d, e):
    n = len(d)
    inp = " ".join([str(n)] + [repr(float(x)) for x in d] + [repr(float(x)) for x in e])
    r = subprocess.run([exe, "leaf"], input=inp, capture_output=True, text=True, env=_env(), timeout=60)
    assert r.returncode == 0, r.stderr[-4000:]
    rows = r.stdout.split("\n")
    st, nrot = (int(x) for x in rows[0].split())
    vals = np.array([[float(x) for x in ln.split()] for ln in rows[1:1 + n]])
    return st, nrot, vals[:, 0], vals[:, 1], vals[:, 2]


@pytest.mark.parametrize("fam", ["uniform", "normal", "toeplitz", "wilkinson", "clustered", "paper_clustered"])
def test_leaf_ql_against_lapack(exe, fam):
    from scipy.linalg import eigh_tridiagonal

    for n in [1, 2, 3, 7, 16, 32, 33, 64]:
        d, e = tdgen.tridiag(fam, n)
        tn = tdgen.tnorm1(d, e)
        st, nrot, lam, r0, r1 = _leaf(exe, d, e)
        assert st == 0
        assert np.all(np.diff(lam) >= 0)
        if n == 1:
            assert lam[0] == d[0] and r0[0] == 1.0 and r1[0] == 1.0
            continue
        ref, Q = eigh_tridiagonal(d, e)
        assert np.abs(lam - ref).max() <= 16 * np.finfo(float).eps * tn * n, (fam, n)
        # rows of an orthogonal matrix: unit norm; entries match LAPACK's up to
        # the column sign where the eigenvalue is well separated
        assert abs(np.dot(r0, r0) - 1.0) <= 1e-13 and abs(np.dot(r1, r1) - 1.0) <= 1e-13
        gap = np.full(n, np.inf)
        gap[:-1] = np.minimum(gap[:-1], np.diff(ref))
        gap[1:] = np.minimum(gap[1:], np.diff(ref))
        with np.errstate(divide="ignore"):
            tol = 1e-12 + 64 * np.finfo(float).eps * tn / gap
        assert np.all(np.abs(np.abs(r0) - np.abs(Q[0])) <= tol), (fam, n)
        assert np.all(np.abs(np.abs(r1) - np.abs(Q[-1])) <= tol), (fam, n)
        assert np.all(np.abs(r0 * r1 - Q[0] * Q[-1]) <= tol), (fam, n)


@pytest.fixture(scope="module")
def br_exe(tmp_path_factory):
    """The host CPU BR baseline (host_br.cpp) built under ASan/UBSan, serial
    (OpenMP pragmas off), driven by tests/host/host_br_check.cpp."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("hostbr") / "host_br_check")
    src = [os.path.join(ROOT, "tests", "host", "host_br_check.cpp"),
           os.path.join(ROOT, "paper_2605_26599_amd", "csrc", "host_br.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", "-o", out] + src
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.mark.parametrize("fam,n", [("uniform", 1), ("uniform", 2), ("uniform", 33), ("normal", 700),
                                   ("toeplitz", 300), ("wilkinson", 129), ("clustered", 500),
                                   ("paper_clustered", 257)])
def test_host_br_sanitized(br_exe, fam, n):
    import oracle

    d, e = tdgen.tridiag(fam, n)
    if fam == "normal":
        e = e.copy()
        e[::50] = 0.0  # blocks through the driver's split
    inp = " ".join([str(n)] + [repr(float(x)) for x in d] + [repr(float(x)) for x in e])
    r = subprocess.run([br_exe], input=inp, capture_output=True, text=True, env=_env(), timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    rows = r.stdout.split()
    assert int(rows[0]) == 0
    lam = np.array([float(x) for x in rows[1:1 + n]])
    assert np.abs(lam - oracle.eigvals(d, e)).max() <= 2e-11 * max(tdgen.tnorm1(d, e), 1e-300)
