"""Benchmark: FP64 tridiagonal eigenvalues/s on one MI355X.

Default workload: one n = 65536 tridiagonal with d, e ~ U(-1, 1) (seeded),
inputs resident in HBM before the timed region.  A step is one full solve
(scale, leaves, every merge level) through the C-ABI.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--family", default="uniform")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--batched", action="store_true", help="4096 problems, log-uniform sizes in [32, 4096]")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return ap.parse_args()


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

    dev = torch.device("cuda:0")
    leaf = args.leaf or None
    if args.batched:
        batch = tdgen.batched(args.family, count=4096, lo=32, hi=4096, inst=0)
        d = torch.from_numpy(batch.d).to(dev)
        e = torch.from_numpy(batch.e).to(dev)
        offs = batch.offsets
        n_total = int(offs[-1])

        def step():
            tde.eigvals_batched(d, e, offs, leaf=leaf, out=out, check=False)

        out = torch.empty(n_total, dtype=torch.float64, device=dev)
        workload = {"workload": f"batched 4096 tridiagonals, sizes log-uniform in [32,4096] (total {n_total}), "
                                f"{args.family}", "problems": 4096, "columns": n_total}
        metric, unit, per_step = "batched solves/s", "solves/s", 4096
    else:
        n = args.n
        dn, en = tdgen.tridiag(args.family, n, cfg=tdgen.CFG_FAMILIES)
        d = torch.from_numpy(dn).to(dev)
        e = torch.from_numpy(en).to(dev)
        out = torch.empty(n, dtype=torch.float64, device=dev)

        def step():
            tde.eigvals(d, e, leaf=leaf, out=out, check=False)

        workload = {"workload": f"single tridiagonal n={n}, {args.family}", "n": n}
        metric, unit, per_step = f"FP64 tridiag eigvals/s @n={n}", "eigvals/s", n

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / args.steps
    value = per_step / (ms / 1e3)
    rec = {
        "metric": metric,
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": workload,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
