"""Binding of libtde_host.so: boundary-row divide and conquer on the host CPU
(the paper's CPU design, Section 4.2), the second host baseline beside the GPU
library.  NumPy in, NumPy out; argument marshalling only.  The GPU entry
points of this package never call it."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtde_host.so")

TDE_HOST_OK = 0
TDE_HOST_EINVAL = -1
TDE_HOST_ENONFINITE = -4
TDE_HOST_ENOCONV = 1
EXPORTS = ("tde_host_workspace", "tde_host_eigvals")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2605_26599_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        i64, i64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.tde_host_workspace.argtypes = [i64, i64p, i64p]
        L.tde_host_workspace.restype = ctypes.c_int
        L.tde_host_eigvals.argtypes = [dp, dp, i64, dp, dp, i64, ctypes.POINTER(ctypes.c_int), i64, ctypes.c_int]
        L.tde_host_eigvals.restype = ctypes.c_int
        _lib = L
    return _lib


def workspace(n: int):
    lw, liw = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib().tde_host_workspace(int(n), ctypes.byref(lw), ctypes.byref(liw))
    if rc != TDE_HOST_OK:
        raise ValueError("tde_host_workspace: bad size")
    return int(lw.value), int(liw.value)


def eigvals(d, e, threads: int = 0, work=None):
    """Ascending eigenvalues of the tridiagonal (d[n], e[n-1]) on the host's
    cores (threads = 0: the OpenMP default).  work: optional preallocated
    (double array, int32 array) of tde_host_workspace's sizes.  Raises on a
    bad argument or non-finite input; a non-converged iteration raises too."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = d.size
    if e.size < max(n - 1, 0):
        raise ValueError("e must hold n-1 entries")
    lam = np.empty(n, dtype=np.float64)
    lw, liw = workspace(n)
    if work is None:
        work = (np.empty(max(lw, 1), dtype=np.float64), np.empty(max(liw, 1), dtype=np.int32))
    w, iw = work
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib().tde_host_eigvals(d.ctypes.data_as(dp), e.ctypes.data_as(dp), n, lam.ctypes.data_as(dp),
                                w.ctypes.data_as(dp), w.size, iw.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                iw.size, int(threads))
    if rc != TDE_HOST_OK:
        raise RuntimeError(f"tde_host_eigvals failed ({rc})")
    return lam
