"""Autotuner for the solver's launch shape.

Knobs that change speed but not the method: the leaf size (largest block of
the merge tree), how leaves are solved (QL, or their own divide and conquer
inside one wave), the target number of poles each lane sweeps in the
root-parallel kernels (which sets the lanes per root, G <= 16, per level),
the number of active roots from which a merge uses the wide sweeps (64 roots
per workgroup, poles split over its waves), and three workgroup-shape knobs:
the most lanes per root in the fused small merges (4, 8, 16, or chosen per
level), the most workgroups of a wide-sweep launch, and the most active roots
one workgroup solves on levels of few merges (larger merges of those levels
go root-parallel).  `tune` times every combination of the first four on the
device (graph replay, inputs resident), then the shape knobs around the
fastest, and keeps the fastest.  Results are
cached in a JSON file keyed by the GPU architecture and a size bucket (log2
of the column count, batch or single), so later runs reuse them without
re-timing.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

LEAVES = (2, 4, 8, 16, 32)     # QL leaves
DC_LEAVES = (32, 64)           # leaves solved by divide and conquer inside one wave
SWEEP_COLS = (8, 16, 32, 64)
WIDE_MIN = (1024, 64, 32)
# (group_max, wide_blocks) tried around the best of the grid above (0 = library default)
SHAPES = ((0, 0), (4, 0), (16, 0), (0, 256), (0, 1024), (4, 256), (16, 256))
# fuse_few tried around the best shape, each with that shape's wide_min and
# with no wide sweeps at all (the merges it hands over then take the
# root-parallel tiles)
FUSE_FEW = (32, 64)
NO_WIDE = 1 << 30


def cache_path() -> str:
    p = os.environ.get("TDE_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "tde", "tuned.json")


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def bucket(n_total: int, batch: int) -> str:
    kind = "batch" if batch > 1 else "single"
    return f"{kind}:2^{max(0, int(math.ceil(math.log2(max(n_total, 1)))))}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(n_total: int, batch: int = 1, device=None):
    """Cached (leaf, sweep_cols, wide_min, leaf_dc, group_max, wide_blocks,
    fuse_few) for this size bucket, or None."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    rec = _load().get(_arch(dev), {}).get(bucket(n_total, batch))
    if rec and "fuse_few" in rec:
        return (int(rec["leaf"]), int(rec["sweep_cols"]), int(rec["wide_min"]), bool(rec["leaf_dc"]),
                int(rec["group_max"]), int(rec["wide_blocks"]), int(rec["fuse_few"]))
    return None


def _time(step, reps: int) -> float:
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        step()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(d: torch.Tensor, e: torch.Tensor, offsets=None, reps: int = 5, leaves=LEAVES, sweep_cols=SWEEP_COLS,
         wide_mins=WIDE_MIN, dc_leaves=DC_LEAVES, shapes=SHAPES, fuse_few=FUSE_FEW, store: bool = True) -> dict:
    """Time every (leaf, leaf solver, sweep_cols, wide_min) on this input, then
    the workgroup-shape knobs (group_max, wide_blocks, then fuse_few) around the
    fastest; return and cache the best.

    d, e are device tensors (single problem: e has n-1 entries; batch: offsets
    is the host offsets sequence).  Returns {"leaf", "leaf_dc", "sweep_cols",
    "wide_min", "group_max", "wide_blocks", "fuse_few", "ms", "table": [(leaf,
    leaf_dc, cols, wide_min, group_max, wide_blocks, fuse_few, ms), ...],
    "tune_s"}.
    """
    import paper_2605_26599_amd as tde

    t0 = time.perf_counter()
    out = torch.empty(d.numel(), dtype=torch.float64, device=d.device)
    table = []

    def run(leaf, dc, cols, wm, gm, wb, ff):
        if offsets is None:
            def step():
                tde.eigvals(d, e, leaf=leaf, leaf_dc=dc, sweep_cols=cols, wide_min=wm, group_max=gm or None,
                            wide_blocks=wb or None, fuse_few=ff or None, out=out, check=False)
        else:
            def step():
                tde.eigvals_batched(d, e, offsets, leaf=leaf, leaf_dc=dc, sweep_cols=cols, wide_min=wm,
                                    group_max=gm or None, wide_blocks=wb or None, fuse_few=ff or None, out=out,
                                    check=False)
        step()
        step()
        table.append((leaf, dc, cols, wm, gm, wb, ff, _time(step, reps)))

    def fastest():
        return min(table, key=lambda r: r[7])

    cands = [(leaf, False) for leaf in leaves] + [(leaf, True) for leaf in dc_leaves]
    for leaf, dc in cands:
        for cols in sweep_cols:
            for wm in wide_mins:
                run(leaf, dc, cols, wm, 0, 0, 0)
    b = fastest()
    for gm, wb in shapes:
        if (gm, wb) != (0, 0):
            run(b[0], b[1], b[2], b[3], gm, wb, 0)
    b = fastest()
    for ff in fuse_few:
        for wm in (b[3], NO_WIDE):
            run(b[0], b[1], b[2], wm, b[4], b[5], ff)
    best = fastest()
    n_total = int(d.numel()) if offsets is None else int(offsets[-1])
    batch = 1 if offsets is None else len(offsets) - 1
    res = {"leaf": best[0], "leaf_dc": best[1], "sweep_cols": best[2], "wide_min": best[3],
           "group_max": best[4], "wide_blocks": best[5], "fuse_few": best[6], "ms": best[7],
           "table": table, "tune_s": time.perf_counter() - t0, "bucket": bucket(n_total, batch)}
    if store:
        db = _load()
        db.setdefault(_arch(d.device), {})[res["bucket"]] = {k: res[k] for k in (
            "leaf", "leaf_dc", "sweep_cols", "wide_min", "group_max", "wide_blocks", "fuse_few", "ms")}
        _store(db)
    return res
