"""Python binding of libtde: FP64 eigenvalues of symmetric tridiagonal matrices
by boundary-row divide and conquer on MI355X (gfx950).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  Importing this
package imports torch first so that libtde binds to the HIP runtime torch has
already loaded (one runtime per process).  There is no CPU fallback: without
the built library or a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

__all__ = [
    "eigvals",
    "eigvals_batched",
    "eigvals_rows",
    "eigvals_selrows",
    "eigvals_noalloc",
    "dense_eigvals",
    "eigvals_ckpt",
    "eigvals_backward",
    "differentiable_eigvals",
    "workspace_bytes",
    "last_status",
    "TDEError",
    "lib",
    "LIB_PATH",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtde.so")

TDE_OK = 0
TDE_EINVAL = -1
TDE_ENOMEM = -2
TDE_EDEVICE = -3
TDE_ENONFINITE = -4
TDE_ENOCONV = 1

EXPORTS = (
    "tde_version",
    "tde_workspace_bytes",
    "tde_eigvals",
    "tde_eigvals_batched",
    "tde_eigvals_rows",
    "tde_eigvals_selrows",
    "tde_selrows_workspace_bytes",
    "tde_eigvals_split",
    "tde_eigvals_noalloc",
    "tde_dense_workspace_bytes",
    "tde_dense_eigvals",
    "tde_checkpoint_bytes",
    "tde_backward_workspace_bytes",
    "tde_eigvals_ckpt",
    "tde_eigvals_backward",
    "tde_get_status",
    "tde_get_counters",
    "tde_timing_enable",
    "tde_timing_read",
    "tde_release_plans",
    "tde_cache_sizes",
    "tde_status_string",
)


class TDEError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _status_string(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class tde_opts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int), ("flags", ctypes.c_int), ("sweep_cols", ctypes.c_int),
                ("wide_min", ctypes.c_int), ("max_sweeps", ctypes.c_int), ("group_max", ctypes.c_int),
                ("wide_blocks", ctypes.c_int), ("fuse_few", ctypes.c_int), ("reserved", ctypes.c_int * 1)]


_lib = None
_lock = threading.Lock()


def _hip_runtimes_loaded():
    libs = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    libs.add(line.split()[-1])
    except OSError:
        pass
    return libs


def lib():
    """Load libtde.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2605_26599_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        optp = ctypes.POINTER(tde_opts)
        L.tde_version.argtypes = []
        L.tde_version.restype = ctypes.c_int
        L.tde_workspace_bytes.argtypes = [i64, i64, optp]
        L.tde_workspace_bytes.restype = sz
        L.tde_eigvals.argtypes = [vp, vp, i64, vp, vp, sz, vp, optp]
        L.tde_eigvals.restype = ctypes.c_int
        L.tde_eigvals_batched.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64), i64, vp, vp, sz, vp, optp]
        L.tde_eigvals_batched.restype = ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.tde_eigvals_rows.argtypes = [vp, vp, i64p, i64, vp, vp, vp, vp, sz, vp, optp]
        L.tde_eigvals_rows.restype = ctypes.c_int
        L.tde_eigvals_split.argtypes = [vp, vp, i64p, i64, vp, vp, sz, vp, optp, i64p]
        L.tde_eigvals_split.restype = ctypes.c_int
        L.tde_checkpoint_bytes.argtypes = [i64p, i64, optp]
        L.tde_checkpoint_bytes.restype = sz
        L.tde_backward_workspace_bytes.argtypes = [i64, i64, optp]
        L.tde_backward_workspace_bytes.restype = sz
        L.tde_eigvals_ckpt.argtypes = [vp, vp, i64p, i64, vp, vp, sz, vp, sz, vp, optp]
        L.tde_eigvals_ckpt.restype = ctypes.c_int
        L.tde_eigvals_backward.argtypes = [vp, vp, i64p, i64, vp, vp, sz, vp, vp, vp, sz, vp, optp]
        L.tde_eigvals_backward.restype = ctypes.c_int
        L.tde_get_status.argtypes = [vp, vp]
        L.tde_get_status.restype = ctypes.c_int
        L.tde_get_counters.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
        L.tde_get_counters.restype = ctypes.c_int
        L.tde_timing_enable.argtypes = [ctypes.c_int]
        L.tde_timing_enable.restype = ctypes.c_int
        L.tde_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.tde_timing_read.restype = ctypes.c_int
        L.tde_release_plans.argtypes = []
        L.tde_release_plans.restype = None
        L.tde_cache_sizes.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.tde_cache_sizes.restype = ctypes.c_int
        L.tde_selrows_workspace_bytes.argtypes = [i64, i64, optp]
        L.tde_selrows_workspace_bytes.restype = sz
        L.tde_eigvals_selrows.argtypes = [vp, vp, i64, i64p, i64, vp, vp, vp, sz, vp, optp]
        L.tde_eigvals_selrows.restype = ctypes.c_int
        L.tde_dense_workspace_bytes.argtypes = [i64, optp]
        L.tde_dense_workspace_bytes.restype = sz
        L.tde_dense_eigvals.argtypes = [vp, i64, i64, vp, vp, vp, vp, sz, vp, optp]
        L.tde_dense_eigvals.restype = ctypes.c_int
        L.tde_eigvals_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, optp]
        L.tde_eigvals_noalloc.restype = ctypes.c_int
        L.tde_status_string.argtypes = [ctypes.c_int]
        L.tde_status_string.restype = ctypes.c_char_p
        _lib = L
        return L


def _status_string(code: int) -> str:
    try:
        return lib().tde_status_string(int(code)).decode()
    except Exception:  # pragma: no cover - only when the library is absent
        return "status"


TDE_FLAG_NO_GRAPH = 1
TDE_FLAG_LEAF_DC = 2


# Schedule options that do not change the method; set_defaults() changes what
# every call below uses when it does not pass them (a tuned choice, say).
# leaf_dc: forward passes solve each leaf by its own divide and conquer inside
# one wave (the reverse mode's checkpointing forward keeps QL leaves).
# max_sweeps: secular iterations allowed per root (a small value forces the
# non-convergence status, for tests).
# group_max: most lanes per root in the fused small merges (4, 8, 16; None = by level).
# wide_blocks: most workgroups of a wide-sweep launch (None = library default).
# fuse_few: on levels of fewer than 1024 merges, the most active roots of a
# merge solved by one workgroup (None = 512); larger ones go root-parallel.
_shape_defaults = {"wide_min": None, "leaf_dc": None, "max_sweeps": None, "group_max": None, "wide_blocks": None,
                   "fuse_few": None}


def set_defaults(wide_min=None, leaf_dc=None, max_sweeps=None, group_max=None, wide_blocks=None, fuse_few=None):
    _shape_defaults["wide_min"] = wide_min
    _shape_defaults["leaf_dc"] = leaf_dc
    _shape_defaults["max_sweeps"] = max_sweeps
    _shape_defaults["group_max"] = group_max
    _shape_defaults["wide_blocks"] = wide_blocks
    _shape_defaults["fuse_few"] = fuse_few


def _opts(leaf, graph=True, sweep_cols=None, wide_min=None, leaf_dc=None, group_max=None, wide_blocks=None,
          fuse_few=None):
    wide_min = _shape_defaults["wide_min"] if wide_min is None else wide_min
    leaf_dc = _shape_defaults["leaf_dc"] if leaf_dc is None else leaf_dc
    group_max = _shape_defaults["group_max"] if group_max is None else group_max
    wide_blocks = _shape_defaults["wide_blocks"] if wide_blocks is None else wide_blocks
    fuse_few = _shape_defaults["fuse_few"] if fuse_few is None else fuse_few
    max_sweeps = _shape_defaults["max_sweeps"]
    if (leaf is None and graph and sweep_cols is None and wide_min is None and not leaf_dc
            and max_sweeps is None and not group_max and not wide_blocks and not fuse_few):
        return None
    o = tde_opts()
    o.leaf = int(leaf or 0)
    o.flags = (0 if graph else TDE_FLAG_NO_GRAPH) | (TDE_FLAG_LEAF_DC if leaf_dc else 0)
    o.sweep_cols = int(sweep_cols or 0)
    o.wide_min = int(wide_min or 0)
    o.max_sweeps = int(max_sweeps or 0)
    o.group_max = int(group_max or 0)
    o.wide_blocks = int(wide_blocks or 0)
    o.fuse_few = int(fuse_few or 0)
    return ctypes.byref(o)


def workspace_bytes(n_total: int, batch: int = 1, leaf=None) -> int:
    nb = int(lib().tde_workspace_bytes(int(n_total), int(batch), _opts(leaf)))
    if nb == 0 and n_total >= 0:
        raise TDEError(TDE_EINVAL, "workspace_bytes")
    return nb


_ws_cache = {}


def _workspace(nbytes: int, device: torch.device) -> torch.Tensor:
    key = (device.index, torch.cuda.current_stream(device).cuda_stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def _check_input(d: torch.Tensor, e: torch.Tensor | None):
    if not isinstance(d, torch.Tensor) or d.dtype != torch.float64 or not d.is_cuda or d.dim() != 1:
        raise TypeError("d must be a 1-D float64 CUDA (HIP) tensor")
    if not d.is_contiguous():
        raise ValueError("d must be contiguous")
    if e is not None:
        if not isinstance(e, torch.Tensor) or e.dtype != torch.float64 or not e.is_cuda or e.dim() != 1:
            raise TypeError("e must be a 1-D float64 CUDA (HIP) tensor")
        if not e.is_contiguous():
            raise ValueError("e must be contiguous")
        if e.device != d.device:
            raise ValueError("d and e must be on the same device")


def eigvals(d: torch.Tensor, e: torch.Tensor, leaf=None, out: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None, check: bool = True, graph: bool = True,
            sweep_cols=None, wide_min=None, leaf_dc=None, group_max=None, wide_blocks=None,
            fuse_few=None) -> torch.Tensor:
    """Eigenvalues (ascending) of the tridiagonal T with diagonal d[n] and
    off-diagonal e[n-1], on d's device and torch's current stream.  graph=True
    replays a captured HIP graph of the whole solve (captured on first use for
    these buffers); graph=False enqueues the kernels one by one.  leaf_dc=True
    solves the leaves by divide and conquer inside one wave each."""
    _check_input(d, e)
    n = d.numel()
    if e.numel() < max(n - 1, 0):
        raise ValueError("e must hold n-1 entries")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=d.device)
    if n == 0:
        return out
    nb = workspace_bytes(n, 1, leaf)
    ws = workspace if workspace is not None else _workspace(nb, d.device)
    if ws.numel() < nb:
        raise ValueError("workspace too small")
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals(d.data_ptr(), e.data_ptr() if e.numel() else None, n, out.data_ptr(),
                               ws.data_ptr(), ws.numel(), stream,
                               _opts(leaf, graph, sweep_cols, wide_min, leaf_dc, group_max, wide_blocks, fuse_few))
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals device status")
    return out


def eigvals_batched(d: torch.Tensor, e: torch.Tensor, offsets, leaf=None, out: torch.Tensor | None = None,
                    workspace: torch.Tensor | None = None, check: bool = True, graph: bool = True,
                    sweep_cols=None, wide_min=None, leaf_dc=None, group_max=None,
                    wide_blocks=None, fuse_few=None) -> torch.Tensor:
    """Eigenvalues of B packed tridiagonals: problem b owns d[offsets[b]:offsets[b+1]]
    and e over the same range (last slot unused).  offsets is a host sequence."""
    _check_input(d, e)
    offs = [int(x) for x in offsets]
    B = len(offs) - 1
    n = offs[-1] if B >= 0 else 0
    if d.numel() < n or e.numel() < n:
        raise ValueError("d and e must hold offsets[-1] entries")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=d.device)
    if B <= 0 or n == 0:
        return out
    nb = workspace_bytes(n, B, leaf)
    ws = workspace if workspace is not None else _workspace(nb, d.device)
    if ws.numel() < nb:
        raise ValueError("workspace too small")
    arr = (ctypes.c_int64 * (B + 1))(*offs)
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_batched(d.data_ptr(), e.data_ptr(), arr, B, out.data_ptr(), ws.data_ptr(),
                                       ws.numel(), stream,
                                       _opts(leaf, graph, sweep_cols, wide_min, leaf_dc, group_max, wide_blocks,
                                             fuse_few))
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals_batched")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals_batched device status")
    return out


def eigvals_noalloc(d: torch.Tensor, e: torch.Tensor, out: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, leaf=None, sweep_cols=None, wide_min=None,
                    leaf_dc=None) -> torch.Tensor:
    """Eigenvalues (ascending) of one tridiagonal of at most 65536 columns,
    through the entry point that allocates no device memory (its workspace is
    a fixed array inside the library, shared by every call on the device:
    calls that overlap on one GPU race).  status, if given, is a device int32
    tensor that receives the solve's device status bits in stream order (0 =
    ok, 1 = non-finite input, 2 or 4 = a leaf or secular iteration hit its
    cap).  Nothing is synchronised."""
    _check_input(d, e)
    n = d.numel()
    if e.numel() < max(n - 1, 0):
        raise ValueError("e must hold n-1 entries")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=d.device)
    if out.dtype != torch.float64 or out.device != d.device or not out.is_contiguous() or out.numel() < n:
        raise ValueError("out must be a contiguous float64 tensor of at least n entries on d's device")
    if status is not None and (status.dtype != torch.int32 or status.device != d.device or status.numel() < 1):
        raise ValueError("status must be an int32 tensor on d's device")
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_noalloc(d.data_ptr(), e.data_ptr() if e.numel() else None, n, out.data_ptr(),
                                       status.data_ptr() if status is not None else None, stream,
                                       _opts(leaf, False, sweep_cols, wide_min, leaf_dc))
    if rc != TDE_OK:
        raise TDEError(rc, "tde_eigvals_noalloc")
    return out


def dense_eigvals(A: torch.Tensor, overwrite: bool = False, leaf=None, sweep_cols=None, wide_min=None,
                  leaf_dc=None, return_tridiagonal: bool = False, check: bool = True):
    """Eigenvalues (ascending) of a dense real symmetric matrix A (n x n float64
    device tensor, both triangles): Householder reduction to tridiagonal form
    on the device, then the boundary-row solve.  A symmetric matrix is its own
    transpose, so torch's row-major storage serves as the column-major input.
    overwrite=False reduces a copy; True lets the reduction destroy A.
    return_tridiagonal=True also returns (d, e) of the reduced matrix."""
    if not isinstance(A, torch.Tensor) or A.dtype != torch.float64 or not A.is_cuda or A.dim() != 2:
        raise TypeError("A must be a 2-D float64 CUDA (HIP) tensor")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    work = A if overwrite else A.clone()
    if not work.is_contiguous():
        raise ValueError("A must be contiguous")
    lam = torch.empty(n, dtype=torch.float64, device=A.device)
    d = torch.empty(n, dtype=torch.float64, device=A.device) if return_tridiagonal else None
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=A.device) if return_tridiagonal else None
    opts = _opts(leaf, True, sweep_cols, wide_min, leaf_dc)
    nb = int(lib().tde_dense_workspace_bytes(n, opts))
    if nb == 0 and n > 0:
        raise TDEError(TDE_EINVAL, "tde_dense_workspace_bytes")
    key = ("dense", A.device.index, torch.cuda.current_stream(A.device).cuda_stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=A.device)
        _ws_cache[key] = ws
    stream = torch.cuda.current_stream(A.device).cuda_stream
    with torch.cuda.device(A.device):
        rc = lib().tde_dense_eigvals(work.data_ptr(), n, n, lam.data_ptr(), d.data_ptr() if d is not None else None,
                                     e.data_ptr() if e is not None else None, ws.data_ptr(), ws.numel(), stream,
                                     opts)
        if rc != TDE_OK:
            raise TDEError(rc, "tde_dense_eigvals")
        if check and n > 0:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_dense_eigvals device status")
    if return_tridiagonal:
        return lam, d, e[:max(n - 1, 0)]
    return lam


# --- driver pre-pass: split at negligible couplings ----------------------------

def eigvals_split(d: torch.Tensor, e: torch.Tensor, offsets=None, leaf=None, sweep_cols=None, check: bool = True,
                  graph: bool = True, wide_min=None, leaf_dc=None):
    """Eigenvalues (ascending per problem) after splitting every problem at its
    negligible couplings (|e_i| <= eps sqrt|d_i d_i+1|) into independently
    scaled blocks.  offsets None = one problem with e[n-1], else the batched
    layout.  Waits for the stream once.  Returns (lam, number of blocks)."""
    _check_input(d, e)
    offs, B, arr = _offsets(d.numel(), offsets)
    n = offs[-1]
    lam = torch.empty(n, dtype=torch.float64, device=d.device)
    if B <= 0 or n == 0:
        return lam, 0
    if d.numel() < n or (offsets is not None and e.numel() < n) or e.numel() < n - 1:
        raise ValueError("d and e are shorter than the offsets require")
    nb = workspace_bytes(n, n, leaf)
    ws = _workspace(nb, d.device)
    nblocks = ctypes.c_int64(0)
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_split(d.data_ptr(), e.data_ptr() if e.numel() else None, arr, B, lam.data_ptr(),
                                     ws.data_ptr(), ws.numel(), stream,
                                     _opts(leaf, graph, sweep_cols, wide_min, leaf_dc), ctypes.byref(nblocks))
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals_split")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals_split device status")
    return lam, int(nblocks.value)


# --- boundary rows at the top (NEXT: requested rows, Golub-Welsch) -----------

def eigvals_rows(d: torch.Tensor, e: torch.Tensor, offsets=None, leaf=None, sweep_cols=None, check: bool = True,
                 graph: bool = True, leaf_dc=None):
    """Eigenvalues (ascending per problem) and, for each, the first and last
    components of its unit eigenvector (first >= 0).  offsets None = one
    problem with e[n-1], else the batched layout.  Returns (lam, qfirst, qlast)."""
    _check_input(d, e)
    offs, B, arr = _offsets(d.numel(), offsets)
    n = offs[-1]
    lam = torch.empty(n, dtype=torch.float64, device=d.device)
    q0 = torch.empty(n, dtype=torch.float64, device=d.device)
    q1 = torch.empty(n, dtype=torch.float64, device=d.device)
    if B <= 0 or n == 0:
        return lam, q0, q1
    if d.numel() < n or (offsets is not None and e.numel() < n) or e.numel() < n - 1:
        raise ValueError("d and e are shorter than the offsets require")
    nb = workspace_bytes(n, B, leaf)
    ws = _workspace(nb, d.device)
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_rows(d.data_ptr(), e.data_ptr() if e.numel() else None, arr, B, lam.data_ptr(),
                                    q0.data_ptr(), q1.data_ptr(), ws.data_ptr(), ws.numel(), stream,
                                    _opts(leaf, graph, sweep_cols, None, leaf_dc))
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals_rows")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals_rows device status")
    return lam, q0, q1


def eigvals_selrows(d: torch.Tensor, e: torch.Tensor, rows, leaf=None, sweep_cols=None, wide_min=None,
                    check: bool = True):
    """Eigenvalues (ascending) of one tridiagonal and the requested rows of its
    eigenvector matrix: Q[i, k] = q_(rows[i]) k, rows in any order with repeats
    allowed, every column signed so that q_0k >= 0 (q_(n-1)k >= 0 when
    q_0k = 0).  Leaves are solved by QL.  Waits for the stream.  Returns
    (lam[n], Q[m, n])."""
    _check_input(d, e)
    n = d.numel()
    if e.numel() < max(n - 1, 0):
        raise ValueError("e must hold n-1 entries")
    rl = [int(r) for r in rows]
    m = len(rl)
    lam = torch.empty(n, dtype=torch.float64, device=d.device)
    Q = torch.empty((m, n), dtype=torch.float64, device=d.device)
    arr = (ctypes.c_int64 * max(m, 1))(*rl)
    opts = _opts(leaf, True, sweep_cols, wide_min)
    nb = int(lib().tde_selrows_workspace_bytes(n, m, opts))
    if nb == 0:
        raise TDEError(TDE_EINVAL, "tde_selrows_workspace_bytes")
    ws = torch.empty(nb, dtype=torch.uint8, device=d.device)
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_selrows(d.data_ptr(), e.data_ptr() if e.numel() else None, n, arr, m,
                                       lam.data_ptr(), Q.data_ptr(), ws.data_ptr(), ws.numel(), stream, opts)
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals_selrows")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals_selrows device status")
    return lam, Q


# --- reverse mode -------------------------------------------------------------

def _offsets(n: int, offsets):
    offs = [0, int(n)] if offsets is None else [int(x) for x in offsets]
    B = len(offs) - 1
    return offs, B, (ctypes.c_int64 * (B + 1))(*offs)


def checkpoint_bytes(n: int, offsets=None, leaf=None, sweep_cols=None) -> int:
    offs, B, arr = _offsets(n, offsets)
    nb = int(lib().tde_checkpoint_bytes(arr, B, _opts(leaf, True, sweep_cols)))
    if nb == 0 and offs[-1] > 0:
        raise TDEError(TDE_EINVAL, "checkpoint_bytes")
    return nb


def eigvals_ckpt(d: torch.Tensor, e: torch.Tensor, offsets=None, leaf=None, sweep_cols=None, out=None,
                 ckpt=None, workspace=None, check: bool = True, graph: bool = True, wide_min=None,
                 group_max=None, wide_blocks=None, fuse_few=None):
    """Eigenvalues as eigvals / eigvals_batched (offsets None = one problem with
    e[n-1]), plus the checkpoint the reverse pass reads.  Returns (lambda, ckpt).
    group_max, wide_blocks and fuse_few are launch-shape options."""
    _check_input(d, e)
    offs, B, arr = _offsets(d.numel(), offsets)
    n = offs[-1]
    if d.numel() < n or (offsets is not None and e.numel() < n) or e.numel() < n - 1:
        raise ValueError("d and e are shorter than the offsets require")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=d.device)
    cb = checkpoint_bytes(n, offsets, leaf, sweep_cols) if n else 0
    if ckpt is None:
        ckpt = torch.empty(max(cb, 256), dtype=torch.uint8, device=d.device)
    if B <= 0 or n == 0:
        return out, ckpt
    if ckpt.numel() < cb:
        raise ValueError("checkpoint buffer too small")
    nb = workspace_bytes(n, B, leaf)
    ws = workspace if workspace is not None else _workspace(nb, d.device)
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_ckpt(d.data_ptr(), e.data_ptr() if e.numel() else None, arr, B, out.data_ptr(),
                                    ckpt.data_ptr(), ckpt.numel(), ws.data_ptr(), ws.numel(), stream,
                                    _opts(leaf, graph, sweep_cols, wide_min, group_max=group_max,
                                          wide_blocks=wide_blocks, fuse_few=fuse_few))
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals_ckpt")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals_ckpt device status")
    return out, ckpt


def eigvals_backward(d: torch.Tensor, e: torch.Tensor, glam: torch.Tensor, ckpt: torch.Tensor, offsets=None,
                     leaf=None, sweep_cols=None, workspace=None, check: bool = True, graph: bool = True,
                     gd: torch.Tensor | None = None, ge: torch.Tensor | None = None, wide_min=None,
                     group_max=None, wide_blocks=None, fuse_few=None):
    """dL/dd and dL/de for L = sum_k glam_k lambda_k, from the checkpoint of
    eigvals_ckpt on the same inputs and options.  Returns (gd[n], ge[n]) with
    ge in the batched layout (the last slot of every problem is 0); gd and ge
    may be given as output buffers of at least n entries."""
    _check_input(d, e)
    offs, B, arr = _offsets(d.numel(), offsets)
    n = offs[-1]
    if gd is None:
        gd = torch.zeros(n, dtype=torch.float64, device=d.device)
    if ge is None:
        ge = torch.zeros(max(n, 1), dtype=torch.float64, device=d.device)
    for t in (gd, ge):
        if t.dtype != torch.float64 or t.device != d.device or not t.is_contiguous() or t.numel() < n:
            raise ValueError("gd and ge must be contiguous float64 tensors of at least n entries on d's device")
    if B <= 0 or n == 0:
        return gd[:n], ge[:n]
    glam = glam.to(device=d.device, dtype=torch.float64).contiguous()
    if glam.numel() != n:
        raise ValueError("glam must hold one entry per eigenvalue")
    nb = int(lib().tde_backward_workspace_bytes(n, B, _opts(leaf, True, sweep_cols)))
    ws = workspace if workspace is not None else _workspace(nb, d.device)
    if ws.numel() < nb:
        raise ValueError("workspace too small")
    stream = torch.cuda.current_stream(d.device).cuda_stream
    with torch.cuda.device(d.device):
        rc = lib().tde_eigvals_backward(d.data_ptr(), e.data_ptr() if e.numel() else None, arr, B,
                                        glam.data_ptr(), ckpt.data_ptr(), ckpt.numel(), gd.data_ptr(),
                                        ge.data_ptr(), ws.data_ptr(), ws.numel(), stream,
                                        _opts(leaf, graph, sweep_cols, wide_min, group_max=group_max,
                                              wide_blocks=wide_blocks, fuse_few=fuse_few))
        if rc != TDE_OK:
            raise TDEError(rc, "tde_eigvals_backward")
        if check:
            st = lib().tde_get_status(ws.data_ptr(), stream)
            if st != TDE_OK:
                raise TDEError(st, "tde_eigvals_backward device status")
    return gd[:n], ge[:n]


class _Eigvals(torch.autograd.Function):
    """lambda(d, e) with the library's reverse pass as its backward."""

    @staticmethod
    def forward(ctx, d, e, offsets, leaf, sweep_cols):
        lam, ckpt = eigvals_ckpt(d, e, offsets, leaf=leaf, sweep_cols=sweep_cols)
        ctx.save_for_backward(d, e, ckpt)
        ctx.cfg = (offsets, leaf, sweep_cols)
        return lam

    @staticmethod
    def backward(ctx, glam):
        d, e, ckpt = ctx.saved_tensors
        offsets, leaf, sweep_cols = ctx.cfg
        gd, ge = eigvals_backward(d, e, glam, ckpt, offsets, leaf=leaf, sweep_cols=sweep_cols)
        gE = torch.zeros_like(e)
        m = min(e.numel(), ge.numel())
        gE[:m] = ge[:m]
        return gd, gE, None, None, None


def differentiable_eigvals(d: torch.Tensor, e: torch.Tensor, offsets=None, leaf=None, sweep_cols=None):
    """Eigenvalues (ascending per problem) as a differentiable function of d and
    e: torch.autograd routes the backward through tde_eigvals_backward.  offsets
    None = one problem (e holds n-1 entries), else the batched layout."""
    offs = None if offsets is None else tuple(int(x) for x in offsets)
    return _Eigvals.apply(d, e, offs, leaf, sweep_cols)


COUNTER_NAMES = ("secular_terms", "lowner_pairs", "row_pairs", "roots", "sweeps", "leaf_columns", "leaf_rotations",
                 "merge_columns", "dc_secular_terms", "dc_lowner_pairs", "dc_row_pairs", "dc_roots",
                 "small_secular_terms", "small_lowner_pairs", "small_row_pairs", "small_roots",
                 "level_secular_terms", "level_lowner_pairs", "level_row_pairs", "level_roots")
KIND_NAMES = ("setup", "leaf", "merge", "deflate", "secular", "lowner", "rows", "assemble", "backward", "small",
              "level")


def counters(workspace: torch.Tensor) -> dict:
    """Algorithmic work counters of the last solve that used this workspace (syncs)."""
    buf = (ctypes.c_uint64 * len(COUNTER_NAMES))()
    stream = torch.cuda.current_stream(workspace.device).cuda_stream
    rc = lib().tde_get_counters(workspace.data_ptr(), stream, buf, len(COUNTER_NAMES))
    if rc != TDE_OK:
        raise TDEError(rc, "tde_get_counters")
    return {name: int(buf[i]) for i, name in enumerate(COUNTER_NAMES)}


def timing_enable(on: bool = True) -> None:
    lib().tde_timing_enable(1 if on else 0)


def timing_read() -> dict:
    """Per launch kind: (milliseconds, launches) recorded since the last read."""
    n = len(KIND_NAMES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    rc = lib().tde_timing_read(ms, cnt, n)
    if rc != TDE_OK:
        raise TDEError(rc, "tde_timing_read")
    return {KIND_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def default_workspace(device=None) -> torch.Tensor:
    """The workspace the convenience functions use on this device and stream."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = (dev.index, torch.cuda.current_stream(dev).cuda_stream)
    return _ws_cache[key]


def cache_sizes() -> dict:
    """Entries in the library's caches: plans, captured graphs, split schedules."""
    buf = (ctypes.c_int64 * 3)()
    rc = lib().tde_cache_sizes(buf, 3)
    if rc != TDE_OK:
        raise TDEError(rc, "tde_cache_sizes")
    return {"plans": int(buf[0]), "graphs": int(buf[1]), "split_schedules": int(buf[2])}


def release_plans() -> None:
    """Free every cached plan, graph and split schedule (waits for their launches)."""
    lib().tde_release_plans()


def last_status(workspace: torch.Tensor) -> int:
    """Device status word of the last solve that used this workspace (syncs)."""
    stream = torch.cuda.current_stream(workspace.device).cuda_stream
    return int(lib().tde_get_status(workspace.data_ptr(), stream))
