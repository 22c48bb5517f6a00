"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/tde.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tde.h")


@pytest.fixture(scope="module")
def L():
    import paper_2605_26599_amd as tde

    if not os.path.exists(tde.LIB_PATH):
        from paper_2605_26599_amd import build

        build.build()
    return tde.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tde_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "tde_eigvals" in names and "tde_eigvals_batched" in names
    for name in names:
        assert hasattr(L, name), name
    import paper_2605_26599_amd as tde

    assert set(names) == set(tde.EXPORTS)


def test_version_and_strings(L):
    assert L.tde_version() >= 100
    assert L.tde_status_string(0) == b"ok"
    assert L.tde_status_string(-1) == b"invalid argument"
    assert L.tde_status_string(1) == b"iteration did not converge"


def test_workspace_is_linear(L):
    import paper_2605_26599_amd as tde

    a = tde.workspace_bytes(1 << 16)
    b = tde.workspace_bytes(1 << 18)
    assert 100 * (1 << 16) < a < 400 * (1 << 16)
    assert abs(b / a - 4.0) < 0.01
    with pytest.raises(tde.TDEError):
        tde.workspace_bytes(100, 1, leaf=65)


def test_argument_errors_are_synchronous(L):
    import paper_2605_26599_amd as tde

    vp = ctypes.c_void_p
    dummy = vp(256)  # never dereferenced: every call below fails its checks first
    assert L.tde_eigvals(dummy, dummy, -1, dummy, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals(dummy, dummy, 0, dummy, dummy, 0, None, None) == tde.TDE_OK
    assert L.tde_eigvals(None, dummy, 10, dummy, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals(dummy, None, 10, dummy, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals(dummy, dummy, 10, dummy, dummy, 16, None, None) == tde.TDE_EINVAL
    bad = tde.tde_opts()
    bad.leaf = 0
    bad.flags = 4  # unknown flag bit
    assert L.tde_eigvals(dummy, dummy, 10, dummy, dummy, 1 << 30, None, ctypes.byref(bad)) == tde.TDE_EINVAL
    for field, value in [("max_sweeps", -1), ("max_sweeps", 97), ("wide_min", 1), ("sweep_cols", -3),
                         ("group_max", 2), ("group_max", 32), ("wide_blocks", -1), ("fuse_few", 1),
                         ("fuse_few", 513), ("fuse_few", -4)]:
        o = tde.tde_opts()
        setattr(o, field, value)
        assert L.tde_eigvals(dummy, dummy, 10, dummy, dummy, 1 << 30, None, ctypes.byref(o)) == tde.TDE_EINVAL, field
    o = tde.tde_opts()
    o.reserved[0] = 7  # reserved fields must be zero
    assert L.tde_eigvals(dummy, dummy, 10, dummy, dummy, 1 << 30, None, ctypes.byref(o)) == tde.TDE_EINVAL
    offs = (ctypes.c_int64 * 3)(0, 5, 3)  # not monotone
    assert L.tde_eigvals_batched(dummy, dummy, offs, 2, dummy, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    offs = (ctypes.c_int64 * 3)(1, 5, 9)  # does not start at 0
    assert L.tde_eigvals_batched(dummy, dummy, offs, 2, dummy, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals_batched(dummy, dummy, None, 2, dummy, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals_batched(dummy, dummy, None, 0, dummy, dummy, 0, None, None) == tde.TDE_OK


def test_checkpoint_and_backward_sizes(L):
    """Host-side size queries of the reverse mode: the checkpoint holds about
    36 bytes per column per tree level, the backward workspace is linear."""
    import paper_2605_26599_amd as tde

    assert tde.checkpoint_bytes(1, leaf=1) >= 256  # no merges: never 0
    for n, leaf, levels in [(8192, 8, 10), (8192, 32, 8), (1000, 1, 10), (33, 32, 1)]:
        nb = tde.checkpoint_bytes(n, leaf=leaf)
        assert 36 * n * levels <= nb <= 36 * n * levels + 8 * 256 + 256, (n, leaf, nb)
    offs = [i * 1024 for i in range(257)]
    assert tde.checkpoint_bytes(offs[-1], offsets=offs, leaf=32) == tde.checkpoint_bytes(
        offs[-1], offsets=[0] + offs[1:], leaf=32)
    a = L.tde_backward_workspace_bytes(1 << 16, 1, None)
    b = L.tde_backward_workspace_bytes(1 << 18, 1, None)
    assert abs(b / a - 4.0) < 0.01 and a > tde.workspace_bytes(1 << 16)
    bad = (ctypes.c_int64 * 3)(0, 5, 3)
    assert L.tde_checkpoint_bytes(bad, 2, None) == 0
    vp = ctypes.c_void_p
    dummy = vp(256)
    offs = (ctypes.c_int64 * 2)(0, 100)
    # missing checkpoint / too small checkpoint / workspace: rejected before any device work
    assert L.tde_eigvals_ckpt(dummy, dummy, offs, 1, dummy, None, 0, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals_ckpt(dummy, dummy, offs, 1, dummy, dummy, 16, dummy, 1 << 30, None, None) == tde.TDE_EINVAL
    assert L.tde_eigvals_backward(dummy, dummy, offs, 1, dummy, dummy, 16, dummy, dummy, dummy, 1 << 30, None,
                                  None) == tde.TDE_EINVAL
    assert L.tde_eigvals_backward(dummy, dummy, offs, 1, None, dummy, 1 << 30, dummy, dummy, dummy, 1 << 30,
                                  None, None) == tde.TDE_EINVAL


def test_cache_sizes_query(L):
    """The cache-size query answers without a device (empty caches here)."""
    import paper_2605_26599_amd as tde

    buf = (ctypes.c_int64 * 3)(-1, -1, -1)
    assert L.tde_cache_sizes(buf, 3) == tde.TDE_OK
    assert list(buf) == [0, 0, 0]
    assert L.tde_cache_sizes(None, 3) == tde.TDE_EINVAL


def test_selrows_sizes_and_argument_errors(L):
    """The requested-rows workspace is linear in n (plus the checkpoint's
    n x levels) and in m; rows outside [0, n) are rejected before any device
    work (the pointers passed are never dereferenced)."""
    import paper_2605_26599_amd as tde

    a = L.tde_selrows_workspace_bytes(1 << 14, 4, None)
    b = L.tde_selrows_workspace_bytes(1 << 14, 4 + (1 << 16), None)
    assert a > tde.workspace_bytes(1 << 14)
    assert b - a >= 4 * (1 << 16)
    fake = ctypes.c_void_p(4096)
    for rows in ([5, 100], [-1], [0, 99, 100]):
        arr = (ctypes.c_int64 * len(rows))(*rows)
        rc = L.tde_eigvals_selrows(fake, fake, 100, arr, len(rows), fake, fake, fake, 1 << 30, None, None)
        assert rc == tde.TDE_EINVAL
    # m > 0 with no row list, and an empty problem with requested rows
    assert L.tde_eigvals_selrows(fake, fake, 100, None, 2, fake, fake, fake, 1 << 30, None, None) == tde.TDE_EINVAL
    arr = (ctypes.c_int64 * 1)(0)
    assert L.tde_eigvals_selrows(fake, fake, 0, arr, 1, fake, fake, fake, 1 << 30, None, None) == tde.TDE_EINVAL
