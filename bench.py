"""Benchmark: FP64 tridiagonal eigenvalues/s on one MI355X.

Default workload: one n = 65536 symmetric tridiagonal with d, e ~ U(-1, 1)
(seeded synthetic input), resident in HBM before the timed region.  A step is
one full solve through the C-ABI: validation/scale, leaves, every merge level
(sort, z, deflation, secular roots, boundary-row propagation, assembly).

Prints one JSON line.  Besides the headline value it carries:
  roofline      the dominant kernel (by time in a second, instrumented timed
                region with HIP events around every launch): algorithmic work
                from the library's counters / measured duration vs. MI355X peak
  cpu_baseline  the CPU oracle (Sturm bisection) on a bounded sample of the
                same matrix, on the host's cores
  secondary     batched solves/s (4096 problems), the QL CPU baseline, and
                the reverse mode: (forward with checkpoint + backward) time over
                plain forward time for L = sum_k w_k lambda_k at n = 8192 and
                at 256 problems of n = 1024 (d, e ~ U(-1, 1))
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E

# Algorithmic work per counted unit ("Roofline accounting").
FLOPS_PER_SEC_TERM = 7      # (D_j - D_o) - tau, 1/del, w*r, t*r, 2 accumulations
FLOPS_PER_LOW_PAIR = 5      # (D_o - D_i) + tau, D_k - D_i, divide, multiply
FLOPS_PER_ROW_PAIR = 9      # (D_i - D_o) - tau, zhat/del, y*y+ss, 2 fused dot updates
FLOPS_PER_LEAF_ROT = 26     # one implicit-QL plane rotation incl. the two tracked rows
BYTES_PER_MERGE_COL = 56    # read lambda, blo, bhi; write D, z, RL, RH
BYTES_PER_ASSEMBLE_COL = 48  # read value + 2 row entries; write lambda, blo, bhi


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--family", default="uniform")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--leaf", type=int, default=0, help="0 = autotuned (or library default with --no-tune)")
    ap.add_argument("--sweep-cols", type=int, default=0, help="0 = autotuned (or library default with --no-tune)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--leaf-dc", action="store_true", help="with --leaf: solve leaves by divide and conquer "
                    "inside one wave")
    ap.add_argument("--wide-min", type=int, default=0, help="active roots from which a merge uses the wide "
                    "secular sweep (0 = library default)")
    ap.add_argument("--batched", action="store_true", help="headline = 4096 problems, log-uniform sizes [32,4096]")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baselines")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, run one plain device-to-device copy of MIB MiB (a kernel of known traffic "
                         "that hardware-counter runs use to scale FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def source_hash():
    """Hash of the device code (kernels and their headers, not the host-side
    launch code): hardware-counter figures stay valid while it is unchanged."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_26599_amd", "csrc")
    for f in ("tde_internal.h", "tde_device.h", "tde_adjoint.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "tde_kernels.hip"), "rb") as fh:
        src = fh.read()
    h.update(src.split(b"// Optional per-kernel timing")[0])
    return h.hexdigest()[:16]


def timed(step, steps):
    import torch

    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def roofline(tde, kinds, cnt, steps):
    """Roofline entry for the kernel kind that took the most time."""
    # the level-wide kernels' share of the work (the fused small-merge kernel
    # counts its own part separately)
    def fused(p):
        return (cnt[p + "secular_terms"] * FLOPS_PER_SEC_TERM + cnt[p + "lowner_pairs"] * FLOPS_PER_LOW_PAIR
                + cnt[p + "row_pairs"] * FLOPS_PER_ROW_PAIR)

    work = {
        "secular": ("alu", (cnt["secular_terms"] - cnt["small_secular_terms"] - cnt["level_secular_terms"])
                    * FLOPS_PER_SEC_TERM),
        "lowner": ("alu", (cnt["lowner_pairs"] - cnt["small_lowner_pairs"] - cnt["level_lowner_pairs"])
                   * FLOPS_PER_LOW_PAIR),
        "rows": ("alu", (cnt["row_pairs"] - cnt["small_row_pairs"] - cnt["level_row_pairs"]) * FLOPS_PER_ROW_PAIR),
        "small": ("alu", fused("small_")),
        "level": ("alu", fused("level_")),
        # QL leaves: rotations; leaves solved by divide and conquer in one wave:
        # the secular, Loewner and row work of their merges
        "leaf": ("alu", cnt["leaf_rotations"] * FLOPS_PER_LEAF_ROT + cnt["dc_secular_terms"] * FLOPS_PER_SEC_TERM
                 + cnt["dc_lowner_pairs"] * FLOPS_PER_LOW_PAIR + cnt["dc_row_pairs"] * FLOPS_PER_ROW_PAIR),
        "merge": ("hbm", None),
        "assemble": ("hbm", None),
    }
    ranked = sorted(((ms, k) for k, (ms, n) in kinds.items() if k in work and n > 0), reverse=True)
    if not ranked:
        return None
    ms, kind = ranked[0]
    launches = kinds[kind][1]
    per_launch_ms = ms / launches
    bound, per_solve = work[kind]
    if bound == "alu":
        achieved = per_solve * steps / (ms * 1e-3) / 1e12
        peak, unit = PEAK_FP64_TFLOPS, "TFLOP/s"
        per_launch = per_solve * steps / launches
    else:
        cols = cnt["merge_columns"]
        per_col = BYTES_PER_MERGE_COL if kind == "merge" else BYTES_PER_ASSEMBLE_COL
        per_solve = cols * per_col
        achieved = per_solve * steps / (ms * 1e-3) / 1e9
        peak, unit = PEAK_HBM_GBS, "GB/s"
        per_launch = per_solve * steps / launches
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            rec = json.load(open(tf)).get(kind)
            if rec and rec.get("source_hash") == source_hash():
                traffic = rec["bytes_per_launch"]
        except (ValueError, KeyError):
            traffic = None
    return {
        "kernel": {"secular": "k_secular", "lowner": "k_lowner", "rows": "k_rows",
                   "leaf": "k_leaf_dc" if cnt["leaf_rotations"] == 0 else "k_leaf", "small": "k_small_merge",
                   "level": "k_level_block",
                   "merge": "k_merge", "assemble": "k_assemble"}[kind],
        "bound": bound,
        "achieved": achieved,
        "peak": peak,
        "unit": unit,
        "frac": achieved / peak,
        "traffic": traffic,
        "launches": launches,
        "avg_launch_us": per_launch_ms * 1e3,
        "work_per_launch": per_launch,
        "time_share": ms / sum(v[0] for v in kinds.values()),
    }


def cpu_baseline(d, e, target_s):
    import numpy as np

    import oracle

    n = len(d)
    g = np.random.default_rng(1)
    probe = np.sort(g.choice(n, 8, replace=False))
    t0 = time.perf_counter()
    oracle.eigvals_index(d, e, probe)
    t_probe = time.perf_counter() - t0
    threads = oracle.num_threads()
    per = t_probe / 8 * min(threads, 8)  # CPU-seconds per eigenvalue (probe ran 8 in parallel)
    m = int(max(threads, min(n, target_s * threads / max(per, 1e-9))))
    ks = np.sort(g.choice(n, m, replace=False))
    t0 = time.perf_counter()
    oracle.eigvals_index(d, e, ks)
    t = time.perf_counter() - t0
    return {"value": m / t, "unit": "eigvals/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} of the {n} eigenvalues (uniformly drawn indices) of the same matrix, "
                      f"Sturm bisection, {t:.1f} s wall"}


def ql_baseline(d, e, target_s):
    import oracle

    n = len(d)
    # implicit QL is sequential and ~n^2: time it on the leading m x m block
    m = min(n, 8192)
    t0 = time.perf_counter()
    oracle.ql_eigvals(d[:m], e[:m - 1])
    t = time.perf_counter() - t0
    return {"value": m / t, "unit": "eigvals/s", "cores": 1, "kind": "implicit QL",
            "sample": f"leading {m} x {m} block of the same matrix, {t:.2f} s"}


def grad_ratio(tde, dev, reps=20):
    """fwd+bwd / fwd for the two gradient workloads (graph replay, inputs,
    weights and every output buffer resident before timing)."""
    import numpy as np
    import torch

    import tdgen
    from paper_2605_26599_amd import autotune

    res = {}
    cases = {"single_n8192": [tdgen.tridiag("uniform", 8192, cfg=tdgen.CFG_GRAD)],
             "batch_256x1024": [tdgen.tridiag("uniform", 1024, cfg=tdgen.CFG_GRAD, inst=b) for b in range(256)]}
    for name, probs in cases.items():
        bt = tdgen.pack(probs)
        offs = None if len(probs) == 1 else [int(x) for x in bt.offsets]
        n = int(bt.offsets[-1])
        d = torch.from_numpy(bt.d).to(dev)
        e = torch.from_numpy(bt.e if offs else probs[0][1]).to(dev)
        w = torch.from_numpy(np.concatenate([tdgen.loss_weights(len(p[0]), inst=i) for i, p in enumerate(probs)])).to(dev)
        out = torch.empty(n, dtype=torch.float64, device=dev)
        gd = torch.empty(n, dtype=torch.float64, device=dev)
        ge = torch.empty(n, dtype=torch.float64, device=dev)
        # the forward alone: its fastest configuration (any leaf solver)
        r = autotune.tune(d, e, offs, reps=3)
        fcfg = dict(leaf=r["leaf"], sweep_cols=r["sweep_cols"], wide_min=r["wide_min"], leaf_dc=r["leaf_dc"])

        def fwd():
            if offs is None:
                tde.eigvals(d, e, out=out, check=False, **fcfg)
            else:
                tde.eigvals_batched(d, e, offs, out=out, check=False, **fcfg)

        # forward with checkpoint + reverse pass: its own fastest configuration
        # (the checkpointing forward always solves leaves by QL)
        def make_fb(leaf, cols, wide):
            ck = torch.empty(tde.checkpoint_bytes(n, offs, leaf, cols), dtype=torch.uint8, device=dev)

            def fb():
                tde.eigvals_ckpt(d, e, offs, leaf=leaf, sweep_cols=cols, wide_min=wide, out=out, ckpt=ck,
                                 check=False)
                tde.eigvals_backward(d, e, w, ck, offs, leaf=leaf, sweep_cols=cols, wide_min=wide, gd=gd, ge=ge,
                                     check=False)
            return fb

        best = None
        for leaf in (4, 8, 16, 32):
            for cols in (16, 64):
                for wide in (1024, 64):
                    fb = make_fb(leaf, cols, wide)
                    fb()
                    fb()
                    t = timed(fb, 3) / 3
                    if best is None or t < best[0]:
                        best = (t, leaf, cols, wide)
        _, bleaf, bcols, bwide = best
        fwdbwd = make_fb(bleaf, bcols, bwide)
        qcfg = dict(leaf=bleaf, sweep_cols=bcols, wide_min=bwide)

        def fwd_same():
            if offs is None:
                tde.eigvals(d, e, out=out, check=False, **qcfg)
            else:
                tde.eigvals_batched(d, e, offs, out=out, check=False, **qcfg)

        for _ in range(3):
            fwd()
            fwd_same()
            fwdbwd()
        torch.cuda.synchronize()
        tf = timed(fwd, reps) / reps
        tfs = timed(fwd_same, reps) / reps
        tfb = timed(fwdbwd, reps) / reps
        res[name] = {"fwd_ms": tf, "fwd_bwd_ms": tfb, "ratio": tfb / tf, "fwd_config": fcfg,
                     "fwd_bwd_config": qcfg, "fwd_same_config_ms": tfs, "ratio_same_config": tfb / tfs}
    return res


def split_prepass(tde, dev, reps=10):
    """Driver pre-pass on a reducible input: n = 65536 uniform with every 97th
    coupling zeroed (676 unreduced blocks), split solve against the plain one
    (both include everything they do; the split one reads back the block
    boundaries once per call)."""
    import torch

    import tdgen

    n = 65536
    d, e = tdgen.tridiag("uniform", n, cfg=tdgen.CFG_FAMILIES)
    e = e.copy()
    e[96::97] = 0.0
    dv = torch.from_numpy(d).to(dev)
    ev = torch.from_numpy(e).to(dev)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    kw = dict(leaf=64, leaf_dc=True)
    nb = tde.eigvals_split(dv, ev, **kw)[1]

    def plain():
        tde.eigvals(dv, ev, out=out, check=False, **kw)

    def split():
        tde.eigvals_split(dv, ev, check=False, **kw)

    for _ in range(2):
        plain()
        split()
    torch.cuda.synchronize()
    tp = timed(plain, reps) / reps
    ts = timed(split, reps) / reps
    return {"workload": "uniform n=65536, every 97th coupling zero", "blocks": nb, "plain_ms": tp,
            "split_ms": ts}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2605_26599_amd as tde
    import tdgen

    from paper_2605_26599_amd import autotune

    dev = torch.device("cuda:0")
    tuning = {}
    if args.wide_min:
        tde.set_defaults(wide_min=args.wide_min)

    def choose(d, e, offs, label):
        """(leaf, sweep_cols, wide_min, leaf_dc): explicit flags, else the autotuner (untimed)."""
        if args.leaf or args.sweep_cols or args.no_tune:
            return args.leaf or None, args.sweep_cols or None, args.wide_min or None, bool(args.leaf_dc)
        r = autotune.tune(d, e, offs, reps=3)
        tuning[label] = {"leaf": r["leaf"], "leaf_dc": r["leaf_dc"], "sweep_cols": r["sweep_cols"],
                         "wide_min": r["wide_min"], "best_ms": r["ms"], "configs_tried": len(r["table"]),
                         "tune_s": r["tune_s"]}
        return r["leaf"], r["sweep_cols"], r["wide_min"], r["leaf_dc"]

    def make_batched():
        batch = tdgen.batched("uniform", count=4096, lo=32, hi=4096, inst=0)
        d = torch.from_numpy(batch.d).to(dev)
        e = torch.from_numpy(batch.e).to(dev)
        out = torch.empty(int(batch.offsets[-1]), dtype=torch.float64, device=dev)
        offs = batch.offsets
        bleaf, bcols, bwide, bdc = choose(d, e, offs, "batched")

        def step():
            tde.eigvals_batched(d, e, offs, leaf=bleaf, sweep_cols=bcols, wide_min=bwide, leaf_dc=bdc, out=out,
                                check=False)

        return batch, step, (bleaf, bcols, bwide, bdc)

    if args.batched:
        batch, step, (leaf, cols, wide, dc) = make_batched()
        n_cols = int(batch.offsets[-1])
        workload = {"workload": f"batched: 4096 tridiagonals, sizes log-uniform in [32,4096] "
                                f"({n_cols} columns), d,e ~ U(-1,1)", "problems": 4096, "columns": n_cols,
                    "leaf": leaf or "default", "leaf_solver": "dc" if dc else "ql",
                    "sweep_cols": cols or "default", "wide_min": wide or "default"}
        metric, unit, per_step = "batched solves/s", "solves/s", 4096
        dn = en = None
    else:
        n = args.n
        dn, en = tdgen.tridiag(args.family, n, cfg=tdgen.CFG_FAMILIES)
        d = torch.from_numpy(dn).to(dev)
        e = torch.from_numpy(en).to(dev)
        out = torch.empty(n, dtype=torch.float64, device=dev)
        n_cols = n
        leaf, cols, wide, dc = choose(d, e, None, "single")

        def step():
            tde.eigvals(d, e, leaf=leaf, sweep_cols=cols, wide_min=wide, leaf_dc=dc, out=out, check=False)

        workload = {"workload": f"single tridiagonal n={n}, family {args.family} (seeded synthetic)", "n": n,
                    "leaf": leaf or "default", "leaf_solver": "dc" if dc else "ql",
                    "sweep_cols": cols or "default", "wide_min": wide or "default"}
        metric, unit, per_step = f"FP64 tridiag eigvals/s @n={n}", "eigvals/s", n

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = tde.last_status(tde.default_workspace(dev))
    if st != tde.TDE_OK:
        raise tde.TDEError(st, "device status after warm-up")

    # timed region: the headline value
    t0 = time.perf_counter()
    total_ms = timed(step, args.steps)
    wall = time.perf_counter() - t0
    ms = total_ms / args.steps
    value = per_step / (ms / 1e3)

    # second timed region: per-kernel durations from HIP events on the solve's stream
    tde.timing_read()
    tde.timing_enable(True)
    timed(step, args.steps)
    tde.timing_enable(False)
    kinds = tde.timing_read()
    cnt = tde.counters(tde.default_workspace(dev))
    roof = roofline(tde, kinds, cnt, args.steps)

    rec = {
        "metric": metric,
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": workload,
        "roofline": roof,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kinds.items()},
        "launches_per_step": sum(v[1] for v in kinds.values()) / args.steps,
        "work_counters_per_step": cnt,
        "wall_s": wall,
    }
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["calibration_copy_bytes"] = int(src.numel() * 8)
        del src, dst
    if not args.no_cpu and dn is not None:
        rec["cpu_baseline"] = cpu_baseline(dn, en, args.cpu_seconds)
    sec = {}
    if not args.no_secondary and not args.batched:
        batch, bstep, _ = make_batched()
        for _ in range(2):
            bstep()
        bms = timed(bstep, 5) / 5
        sec["batched_solves_per_s"] = 4096 / (bms / 1e3)
        sec["batched_ms_per_step"] = bms
        sec["grad_fwd_bwd_over_fwd"] = grad_ratio(tde, dev)
        sec["split_prepass"] = split_prepass(tde, dev)
    if not args.no_cpu and dn is not None:
        sec["cpu_ql"] = ql_baseline(dn, en, args.cpu_seconds)
    if sec:
        rec["secondary"] = sec
    if tuning:
        rec["autotune"] = tuning
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
