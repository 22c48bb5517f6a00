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

# Algorithmic work per counted unit, the pass-count model's figures (a divide
# counted as one flop): a secular pole term is a subtraction, a divide, a
# multiply, an add and a fused multiply-add; a Loewner (pole, root) factor is a
# difference and its ratio into the product chain; a boundary-row (root, pole)
# pair is the denominator, the ratio, the norm update and two dot updates.
FLOPS_PER_SEC_TERM = 6
FLOPS_PER_LOW_PAIR = 3
FLOPS_PER_ROW_PAIR = 8
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
    ap.add_argument("--group-max", type=int, default=0, help="most lanes per root in the fused small merges "
                    "(4, 8, 16; 0 = by level)")
    ap.add_argument("--wide-blocks", type=int, default=0, help="most workgroups of a wide-sweep launch "
                    "(0 = library default)")
    ap.add_argument("--fuse-few", type=int, default=0, help="on levels of few merges, the most active roots "
                    "one workgroup solves (0 = library default, 512)")
    ap.add_argument("--wide-min", type=int, default=0, help="active roots from which a merge uses the wide "
                    "secular sweep (0 = library default)")
    ap.add_argument("--batched", action="store_true", help="headline = 4096 problems, log-uniform sizes [32,4096]")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baselines")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--grad", choices=("single", "batch"), default=None,
                    help="time (and let a profiler see) only the reverse-mode step of one gradient workload: "
                         "checkpointing forward + backward, n = 8192 or 256 x 1024, with --leaf, --sweep-cols "
                         "and --wide-min (defaults 8, 16, 1024)")
    ap.add_argument("--dense", type=int, default=0, metavar="N",
                    help="time only the dense front end (reduction + solve) on an N x N matrix")
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


def kind_work(cnt):
    """Algorithmic work per solve of each launch kind: (bound, flops or None)."""
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
    return work


def _profile_record(name, kernel):
    """A hardware-counter record of profiles/<name> for kernel, if it was taken
    from the current kernel sources."""
    tf = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(tf):
        return None
    try:
        db = json.load(open(tf))
    except ValueError:
        return None
    if db.get("source_hash") != source_hash():
        return None
    return db.get("kernels", {}).get(kernel)


def roofline(tde, kinds, cnt, steps, fp64_profile="fp64_uniform_n65536.json", kind=None):
    """Roofline entry for the kernel kind that took the most time (or `kind`)."""
    work = kind_work(cnt)
    ranked = sorted(((ms, k) for k, (ms, n) in kinds.items() if k in work and n > 0), reverse=True)
    if not ranked:
        return None
    if kind is None:
        ms, kind = ranked[0]
    else:
        ms = kinds[kind][0]
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
    kname = {"secular": "k_secular", "lowner": "k_lowner", "rows": "k_rows",
             "leaf": "k_leaf_dc" if cnt["leaf_rotations"] == 0 else "k_leaf", "small": "k_small_merge",
             "level": "k_level_block", "merge": "k_merge", "assemble": "k_assemble"}[kind]
    hw = None
    if bound == "alu":
        # hardware-counted FP64 rate: the profile's FP64 instruction count per
        # launch of this kernel (rocprofv3 SQ_INSTS_VALU_*_F64, same workload
        # and launch configuration) over the live average launch duration
        for k in ((kname + "_wide", kname) if kind in ("secular", "lowner", "rows") else (kname,)):
            rec = _profile_record(fp64_profile, k)
            if rec:
                hw_t = rec["hw_flops_per_launch"] / (per_launch_ms * 1e-3) / 1e12
                hw = {"kernel": k, "profile": "profiles/" + fp64_profile.replace(".json", ".md"),
                      "hw_flops_per_launch": rec["hw_flops_per_launch"], "hw_achieved": hw_t,
                      "hw_frac": hw_t / PEAK_FP64_TFLOPS, "profiled_avg_us": rec["avg_us"]}
                break
    return {
        "kernel": kname,
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
        "flops_per_unit": {"secular_term": FLOPS_PER_SEC_TERM, "lowner_pair": FLOPS_PER_LOW_PAIR,
                           "row_pair": FLOPS_PER_ROW_PAIR},
        "hw_counted": hw,
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, e, target_s):
    """The oracle on a bounded sample of the eigenvalue indices (always
    including the two extreme ones); returns (record, indices, eigenvalues)."""
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
    ks = np.unique(np.concatenate([g.choice(n, m, replace=False), [0, n - 1]]))
    m = len(ks)
    t0 = time.perf_counter()
    lam = oracle.eigvals_index(d, e, ks)
    t = time.perf_counter() - t0
    rec = {"value": m / t, "unit": "eigvals/s", "cores": threads, "kind": "oracle",
           "sample": f"{m} of the {n} eigenvalues (uniformly drawn indices plus the two extreme ones) of the "
                     f"same matrix, Sturm bisection, {t:.1f} s wall", "cpu_model": cpu_model()}
    return rec, ks, lam


def host_br_baseline(d, e, lam_gpu):
    """The host CPU BR baseline (libtde_host.so, the paper's CPU design) on
    the same matrix on every host core: best of 3 wall times, and its largest
    difference from the GPU result."""
    import numpy as np

    from paper_2605_26599_amd import host_br

    n = len(d)
    lw, liw = host_br.workspace(n)
    work = (np.empty(lw), np.empty(liw, dtype=np.int32))
    threads = len(os.sched_getaffinity(0))
    ts = []
    lam = None
    for _ in range(3):
        t0 = time.perf_counter()
        lam = host_br.eigvals(d, e, threads=threads, work=work)
        ts.append(time.perf_counter() - t0)
    t = min(ts)
    return {"value": n / t, "unit": "eigvals/s", "cores": threads, "kind": "host BR D&C (OpenMP)",
            "ms": t * 1e3, "sample": "the whole matrix, best of 3", "cpu_model": cpu_model(),
            "workspace_bytes": 8 * lw + 4 * liw,
            "max_abs_diff_vs_gpu": float(np.abs(lam - np.asarray(lam_gpu)).max())}


def accuracy(lam_gpu, lam_ref, tnorm, lam_inf):
    """The paper's normalised accuracy metrics (Section 5.1): e_fwd =
    ||dlambda||_inf / max(1, ||lambda||_inf), e_bwd = ||dlambda||_inf /
    max(1, ||T||_inf), and the absolute gap in units of ||T||_1."""
    import numpy as np

    err = float(np.abs(np.asarray(lam_gpu) - np.asarray(lam_ref)).max())
    return {"max_abs_err": err, "e_fwd": err / max(1.0, lam_inf), "e_bwd": err / max(1.0, tnorm),
            "err_over_tnorm": err / tnorm, "gate_over_tnorm": 2e-11}


def ql_baseline(d, e):
    """Implicit QL on one core.  It is sequential and ~n^2, so it runs on the
    leading 8192 and 16384 blocks of the same matrix and the time at n is
    extrapolated with the exponent those two points give (labelled so)."""
    import math

    import oracle

    n = len(d)
    pts = []
    for m in sorted({min(n, 8192), min(n, 16384)}):
        t0 = time.perf_counter()
        oracle.ql_eigvals(d[:m], e[:m - 1])
        pts.append((m, time.perf_counter() - t0))
    if pts[-1][0] == n:
        return {"value": n / pts[-1][1], "unit": "eigvals/s", "cores": 1, "kind": "implicit QL",
                "sample": f"the whole matrix, {pts[-1][1]:.2f} s", "extrapolated": False}
    (m1, t1), (m2, t2) = pts[0], pts[-1]
    p = math.log(t2 / t1) / math.log(m2 / m1)
    tn = t2 * (n / m2) ** p
    return {"value": n / tn, "unit": "eigvals/s", "cores": 1, "kind": "implicit QL", "extrapolated": True,
            "sample": f"leading {m1} and {m2} blocks of the same matrix measured ({t1:.2f} s, {t2:.2f} s); "
                      f"time at n={n} extrapolated as t ~ n^{p:.2f}: {tn:.1f} s",
            "measured": [{"n": m1, "s": t1}, {"n": m2, "s": t2}], "exponent": p}


def grad_case(tde, dev, name):
    """Device inputs of one gradient workload: (d, e, w, offsets or None, n)."""
    import numpy as np
    import torch

    import tdgen

    probs = ([tdgen.tridiag("uniform", 8192, cfg=tdgen.CFG_GRAD)] if name.startswith("single") else
             [tdgen.tridiag("uniform", 1024, cfg=tdgen.CFG_GRAD, inst=b) for b in range(256)])
    bt = tdgen.pack(probs)
    offs = None if len(probs) == 1 else [int(x) for x in bt.offsets]
    n = int(bt.offsets[-1])
    d = torch.from_numpy(bt.d).to(dev)
    e = torch.from_numpy(bt.e if offs else probs[0][1]).to(dev)
    w = torch.from_numpy(np.concatenate([tdgen.loss_weights(len(p[0]), inst=i) for i, p in enumerate(probs)])).to(dev)
    return d, e, w, offs, n


def make_fwdbwd(tde, dev, d, e, w, offs, n, leaf, cols, wide, wblocks=None, gmax=None, ffew=None):
    """Checkpointing forward + backward step (all buffers resident)."""
    import torch

    out = torch.empty(n, dtype=torch.float64, device=dev)
    gd = torch.empty(n, dtype=torch.float64, device=dev)
    ge = torch.empty(n, dtype=torch.float64, device=dev)
    ck = torch.empty(tde.checkpoint_bytes(n, offs, leaf, cols), dtype=torch.uint8, device=dev)

    def fb():
        tde.eigvals_ckpt(d, e, offs, leaf=leaf, sweep_cols=cols, wide_min=wide, wide_blocks=wblocks,
                         group_max=gmax, fuse_few=ffew, out=out, ckpt=ck, check=False)
        tde.eigvals_backward(d, e, w, ck, offs, leaf=leaf, sweep_cols=cols, wide_min=wide, wide_blocks=wblocks,
                             group_max=gmax, fuse_few=ffew, gd=gd, ge=ge, check=False)
    return fb


def grad_only(args):
    """--grad: time only the reverse-mode step of one gradient workload."""
    import torch

    import paper_2605_26599_amd as tde

    dev = torch.device("cuda:0")
    d, e, w, offs, n = grad_case(tde, dev, args.grad)
    leaf, cols, wide = args.leaf or 8, args.sweep_cols or 16, args.wide_min or 1024
    fb = make_fwdbwd(tde, dev, d, e, w, offs, n, leaf, cols, wide, args.wide_blocks or None, args.group_max or None,
                     args.fuse_few or None)
    for _ in range(max(args.warmup, 1)):
        fb()
    torch.cuda.synchronize()
    ms = timed(fb, args.steps) / args.steps
    print(json.dumps({"metric": "fwd+bwd ms", "value": ms, "unit": "ms", "steps": args.steps,
                      "higher_is_better": False,
                      "config": {"workload": f"gradient {args.grad}", "leaf": leaf, "sweep_cols": cols,
                                 "wide_min": wide, "wide_blocks": args.wide_blocks or None,
                                 "group_max": args.group_max or None, "fuse_few": args.fuse_few or None}}),
          flush=True)


def grad_ratio(tde, dev, reps=20):
    """fwd+bwd / fwd for the two gradient workloads (graph replay, inputs,
    weights and every output buffer resident before timing)."""
    import torch

    from paper_2605_26599_amd import autotune

    res = {}
    for name in ("single_n8192", "batch_256x1024"):
        d, e, w, offs, n = grad_case(tde, dev, name)
        out = torch.empty(n, dtype=torch.float64, device=dev)
        # the forward alone: its fastest configuration (any leaf solver)
        r = autotune.tune(d, e, offs, reps=3)
        fcfg = dict(leaf=r["leaf"], sweep_cols=r["sweep_cols"], wide_min=r["wide_min"], leaf_dc=r["leaf_dc"],
                    group_max=r["group_max"] or None, wide_blocks=r["wide_blocks"] or None,
                    fuse_few=r["fuse_few"] or None)

        def fwd():
            if offs is None:
                tde.eigvals(d, e, out=out, check=False, **fcfg)
            else:
                tde.eigvals_batched(d, e, offs, out=out, check=False, **fcfg)

        # forward with checkpoint + reverse pass: its own fastest configuration
        best = None
        for leaf in (4, 8, 16, 32):
            for cols in (16, 64):
                for wide in (1024, 64):
                    for wb in (None, 256):
                        for ff in (None, 32):
                            fb = make_fwdbwd(tde, dev, d, e, w, offs, n, leaf, cols, wide, wb, None, ff)
                            fb()
                            fb()
                            t = timed(fb, 3) / 3
                            if best is None or t < best[0]:
                                best = (t, leaf, cols, wide, wb, ff)
        _, bleaf, bcols, bwide, bwb, bff = best
        fwdbwd = make_fwdbwd(tde, dev, d, e, w, offs, n, bleaf, bcols, bwide, bwb, None, bff)
        qcfg = dict(leaf=bleaf, sweep_cols=bcols, wide_min=bwide, wide_blocks=bwb, fuse_few=bff)

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


def _runs(step, warm=2, reps=5):
    """Two warm-ups and five individually timed runs: (median ms, min ms)."""
    import torch

    for _ in range(warm):
        step()
    ts = []
    for _ in range(reps):
        ts.append(timed(step, 1))
    ts.sort()
    return ts[len(ts) // 2], ts[0]


# Launch configurations each secondary workload is timed with (the best is
# reported with its configuration): in-wave leaves of 64 with three sweep
# shapes (one with a small wide-sweep grid), and QL leaves of 32.
SECONDARY_CFGS = ({"leaf": 64, "leaf_dc": True, "sweep_cols": 32, "wide_min": 32},
                  {"leaf": 64, "leaf_dc": True, "sweep_cols": 16, "wide_min": 64},
                  {"leaf": 64, "leaf_dc": True, "sweep_cols": 16, "wide_min": 64, "wide_blocks": 256},
                  {"leaf": 64, "leaf_dc": True, "sweep_cols": 16, "wide_min": 1024, "fuse_few": 32},
                  {"leaf": 64, "leaf_dc": True, "sweep_cols": 64, "wide_min": 32},
                  {"leaf": 32, "leaf_dc": False, "sweep_cols": 32, "wide_min": 32})


def configs_record(tde, dev):
    """Times of the other benchmark workloads in the same run: n = 1024 with
    the prescribed leaf-32 QL solve (20 instances), the four families at
    16384/32768/65536, N(0,1) at 131072 and 262144, Toeplitz at 262144 (each
    with its best of SECONDARY_CFGS), the peak device bytes at 262144, and
    the accuracy metrics where a reference is cheap (the oracle at n = 1024,
    the closed form for Toeplitz)."""
    import math

    import numpy as np
    import torch

    import oracle
    import tdgen

    out = {}

    def solve_fn(dv, ev, o, cfg):
        def step():
            tde.eigvals(dv, ev, out=o, check=False, **cfg)
        return step

    def best_of(dv, ev, o, cfgs=SECONDARY_CFGS):
        best = None
        for cfg in cfgs:
            step = solve_fn(dv, ev, o, cfg)
            step()
            t = timed(step, 2) / 2
            if best is None or t < best[0]:
                best = (t, cfg)
        step = solve_fn(dv, ev, o, best[1])
        med, mn = _runs(step)
        st = tde.last_status(tde.default_workspace(dev))
        if st != tde.TDE_OK:
            raise tde.TDEError(st, "device status")
        return med, mn, best[1]

    # C1: n = 1024, leaf 32 solved by QL (the prescribed configuration), 20 instances
    c1 = {"ms_median": [], "acc": []}
    for inst in range(20):
        d, e = tdgen.tridiag("uniform", 1024, cfg=tdgen.CFG_SMALL, inst=inst)
        dv, ev = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
        o = torch.empty(1024, dtype=torch.float64, device=dev)
        step = solve_fn(dv, ev, o, {"leaf": 32, "leaf_dc": False})
        med, _ = _runs(step)
        c1["ms_median"].append(med)
        ref = oracle.eigvals(d, e)
        c1["acc"].append(accuracy(o.cpu().numpy(), ref, tdgen.tnorm1(d, e), float(np.abs(ref).max())))
    msm = float(np.median(c1["ms_median"]))
    out["c1_uniform_n1024_leaf32_ql"] = {
        "ms_median": msm, "eigvals_per_s": 1024 / (msm / 1e3), "instances": 20,
        "e_fwd_max": max(a["e_fwd"] for a in c1["acc"]), "e_bwd_max": max(a["e_bwd"] for a in c1["acc"]),
        "err_over_tnorm_max": max(a["err_over_tnorm"] for a in c1["acc"]), "reference": "oracle, every eigenvalue"}

    def one(fam, n, cfg_id):
        d, e = tdgen.tridiag(fam, n, cfg=cfg_id)
        dv, ev = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
        o = torch.empty(n, dtype=torch.float64, device=dev)
        med, mn, cfg = best_of(dv, ev, o)
        rec = {"ms_median": med, "ms_min": mn, "eigvals_per_s": n / (med / 1e3), "config": cfg}
        if fam == "toeplitz":
            k = np.arange(1, n + 1, dtype=np.float64)
            ref = np.sort(2.0 - 2.0 * np.cos(k * math.pi / (n + 1)))
            acc = accuracy(o.cpu().numpy(), ref, tdgen.tnorm1(d, e), float(np.abs(ref).max()))
            rec.update({"e_fwd": acc["e_fwd"], "e_bwd": acc["e_bwd"], "err_over_tnorm": acc["err_over_tnorm"],
                        "reference": "closed form 2 - 2 cos(k pi/(n+1)), every eigenvalue"})
        return rec

    for fam in ("uniform", "toeplitz", "wilkinson", "clustered"):
        for n in (16384, 32768, 65536):
            out[f"c2_{fam}_n{n}"] = one(fam, n, tdgen.CFG_FAMILIES)
    for n in (131072, 262144):
        out[f"c3_normal_n{n}"] = one("normal", n, tdgen.CFG_LARGE)
    out["c3_toeplitz_n262144"] = one("toeplitz", 262144, tdgen.CFG_LARGE)

    # peak device bytes of a solve at n = 262144: free device memory before
    # and after inputs, output, workspace and the library's plan tables (and
    # its captured graph) exist, against the workspace query
    n = 262144
    d, e = tdgen.tridiag("normal", n, cfg=tdgen.CFG_LARGE)
    cfg = out["c3_normal_n262144"]["config"]
    tde.release_plans()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info(dev)[0]
    dv, ev = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
    o = torch.empty(n, dtype=torch.float64, device=dev)
    wsb = tde.workspace_bytes(n, 1, cfg["leaf"])
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    tde.eigvals(dv, ev, out=o, workspace=ws, **cfg)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(dev)[0]
    out["c3_device_bytes_n262144"] = {
        "measured_bytes": int(free0 - free1), "bytes_per_column": (free0 - free1) / n,
        "workspace_query_bytes": int(wsb), "inputs_output_bytes": int(8 * (3 * n - 1)),
        "dense_q_bytes": int(8 * n * n),
        "method": "drop in free device memory (hipMemGetInfo) from before the inputs exist to after one solve: "
                  "inputs, output, workspace, plan tables and the captured graph (torch rounds its blocks up)"}
    del dv, ev, o, ws
    torch.cuda.empty_cache()
    return out


def toeplitz_roofline(tde, dev, cfg, steps=5):
    """Roofline of the wide secular sweep on the large merges: Toeplitz
    n = 65536 (half of every merge's columns stay active), with per-launch
    times from HIP events on the solve's stream."""
    import torch

    import tdgen

    n = 65536
    d, e = tdgen.tridiag("toeplitz", n, cfg=tdgen.CFG_FAMILIES)
    dv, ev = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
    o = torch.empty(n, dtype=torch.float64, device=dev)

    def step():
        tde.eigvals(dv, ev, out=o, check=False, **cfg)

    step()
    torch.cuda.synchronize()
    tde.timing_read()
    tde.timing_enable(True)
    timed(step, steps)
    tde.timing_enable(False)
    kinds = tde.timing_read()
    cnt = tde.counters(tde.default_workspace(dev))
    r = roofline(tde, kinds, cnt, steps, fp64_profile="fp64_toeplitz_n65536.json", kind="secular")
    r["workload"] = "Toeplitz n=65536 (d=2, e=-1)"
    r["config"] = cfg
    r["mean_sweeps_per_root"] = cnt["sweeps"] / max(cnt["roots"], 1)
    return r


def dense_record(tde, dev, n=4096, reps=3):
    """Dense front end on a matrix with a prescribed spectrum: A = Q diag(lambda)
    Q^T, Q a seeded random orthogonal matrix, lambda ~ U(-1, 1); Householder
    reduction on the device plus the boundary-row solve.  Each timed step
    starts from a fresh device copy of A (the reduction destroys it); the copy
    is timed alone and subtracted.  The trailing-matrix products of the
    reduction read sum_c 8 (n - c - 1)^2 bytes, the figure its HBM rate uses."""
    import numpy as np
    import torch

    g = np.random.default_rng(np.random.SeedSequence([2605, 26599, 6, n]))
    Q, R = np.linalg.qr(g.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))[None, :]
    lam = np.sort(g.uniform(-1.0, 1.0, n))
    A = Q @ (lam[:, None] * Q.T)
    A = 0.5 * (A + A.T)
    src = torch.from_numpy(A).to(dev)
    work = torch.empty_like(src)

    def copy():
        work.copy_(src)

    def solve():
        work.copy_(src)
        tde.dense_eigvals(work, overwrite=True, check=False)

    solve()
    torch.cuda.synchronize()
    out = tde.dense_eigvals(src.clone(), overwrite=True).cpu().numpy()
    tc = timed(copy, reps) / reps
    ts = timed(solve, reps) / reps - tc
    # the tridiagonal solve alone on the reduced (d, e)
    _, d, e = tde.dense_eigvals(src.clone(), overwrite=True, return_tridiagonal=True)
    o = torch.empty(n, dtype=torch.float64, device=dev)

    def tri():
        tde.eigvals(d, e, out=o, check=False)

    tri()
    tt = timed(tri, reps) / reps
    m = np.arange(n - 2, 0, -1, dtype=np.float64)
    sym_bytes = float(8.0 * np.sum(m * m))
    err = float(np.abs(out - lam).max())
    norm1 = float(np.abs(A).sum(axis=0).max())
    return {"workload": f"dense symmetric n={n}, prescribed spectrum U(-1,1), seeded random orthogonal Q",
            "ms": ts, "eigvals_per_s": n / (ts / 1e3), "tridiagonal_solve_ms": tt, "reduction_ms": ts - tt,
            "trailing_product_bytes": sym_bytes, "reduction_hbm_gbs_lower_bound": sym_bytes / ((ts - tt) * 1e-3) / 1e9,
            "max_abs_err_vs_prescribed": err, "err_over_norm1": err / norm1, "gate_over_norm1": 2e-11}


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
    if args.grad:
        grad_only(args)
        return
    if args.dense:
        import torch

        import paper_2605_26599_amd as tde

        print(json.dumps(dense_record(tde, torch.device("cuda:0"), n=args.dense, reps=max(args.steps, 1))),
              flush=True)
        return
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
        """Launch options: explicit flags, else the autotuner (untimed)."""
        if args.leaf or args.sweep_cols or args.no_tune:
            return {"leaf": args.leaf or None, "sweep_cols": args.sweep_cols or None,
                    "wide_min": args.wide_min or None, "leaf_dc": bool(args.leaf_dc),
                    "group_max": args.group_max or None, "wide_blocks": args.wide_blocks or None,
                    "fuse_few": args.fuse_few or None}
        r = autotune.tune(d, e, offs, reps=3)
        tuning[label] = {"leaf": r["leaf"], "leaf_dc": r["leaf_dc"], "sweep_cols": r["sweep_cols"],
                         "wide_min": r["wide_min"], "group_max": r["group_max"], "wide_blocks": r["wide_blocks"],
                         "fuse_few": r["fuse_few"], "best_ms": r["ms"], "configs_tried": len(r["table"]),
                         "tune_s": r["tune_s"]}
        return {"leaf": r["leaf"], "sweep_cols": r["sweep_cols"], "wide_min": r["wide_min"], "leaf_dc": r["leaf_dc"],
                "group_max": r["group_max"] or None, "wide_blocks": r["wide_blocks"] or None,
                "fuse_few": r["fuse_few"] or None}

    def describe(cfg):
        return {"leaf": cfg["leaf"] or "default", "leaf_solver": "dc" if cfg["leaf_dc"] else "ql",
                "sweep_cols": cfg["sweep_cols"] or "default", "wide_min": cfg["wide_min"] or "default",
                "group_max": cfg["group_max"] or "by level", "wide_blocks": cfg["wide_blocks"] or "default",
                "fuse_few": cfg["fuse_few"] or "default"}

    def make_batched():
        batch = tdgen.batched("uniform", count=4096, lo=32, hi=4096, inst=0)
        d = torch.from_numpy(batch.d).to(dev)
        e = torch.from_numpy(batch.e).to(dev)
        out = torch.empty(int(batch.offsets[-1]), dtype=torch.float64, device=dev)
        offs = batch.offsets
        bcfg = choose(d, e, offs, "batched")

        def step():
            tde.eigvals_batched(d, e, offs, out=out, check=False, **bcfg)

        return batch, step, bcfg

    if args.batched:
        batch, step, cfg = make_batched()
        n_cols = int(batch.offsets[-1])
        workload = {"workload": f"batched: 4096 tridiagonals, sizes log-uniform in [32,4096] "
                                f"({n_cols} columns), d,e ~ U(-1,1)", "problems": 4096, "columns": n_cols,
                    **describe(cfg)}
        metric, unit, per_step = "batched solves/s", "solves/s", 4096
        dn = en = None
    else:
        n = args.n
        dn, en = tdgen.tridiag(args.family, n, cfg=tdgen.CFG_FAMILIES)
        d = torch.from_numpy(dn).to(dev)
        e = torch.from_numpy(en).to(dev)
        out = torch.empty(n, dtype=torch.float64, device=dev)
        n_cols = n
        cfg = choose(d, e, None, "single")

        def step():
            tde.eigvals(d, e, out=out, check=False, **cfg)

        workload = {"workload": f"single tridiagonal n={n}, family {args.family} (seeded synthetic)", "n": n,
                    **describe(cfg)}
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
    prof = f"fp64_{'batched_4096' if args.batched else f'{args.family}_n{args.n}'}.json"
    roof = roofline(tde, kinds, cnt, args.steps, fp64_profile=prof)

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
        "launches_per_step_by_kind": {k: v[1] / args.steps for k, v in kinds.items() if v[1]},
        "work_flops_per_step": {k: w for k, (b, w) in kind_work(cnt).items() if w is not None},
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
        cb, ks, lam_ref = cpu_baseline(dn, en, args.cpu_seconds)
        rec["cpu_baseline"] = cb
        # accuracy of the timed solve on the oracle's sampled indices (the two
        # extreme eigenvalues included, so ||lambda||_inf is exact)
        rec["accuracy"] = accuracy(out.cpu().numpy()[ks], lam_ref, tdgen.tnorm1(dn, en),
                                   float(np.abs(lam_ref).max()))
        rec["accuracy"]["sample"] = f"{len(ks)} oracle eigenvalues (the cpu_baseline sample)"
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
        sec["dense_front_end"] = dense_record(tde, dev)
        sec["configs"] = configs_record(tde, dev)
        sec["toeplitz_roofline"] = toeplitz_roofline(tde, dev, sec["configs"]["c2_toeplitz_n65536"]["config"])
    if not args.no_cpu and dn is not None:
        sec["cpu_br"] = host_br_baseline(dn, en, out.cpu().numpy())
        sec["cpu_ql"] = ql_baseline(dn, en)
    if sec:
        rec["secondary"] = sec
    if tuning:
        rec["autotune"] = tuning
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
