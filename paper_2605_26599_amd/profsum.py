"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2605_26599_amd.profsum stats  <kernel_stats.csv> <bench.jsonl> <out.md> <title> <command>
  python -m paper_2605_26599_amd.profsum traffic <fetch_counter.csv> <write_counter.csv> <copy_bytes> <out.json> <out.md> <command> [<kernel_trace.csv>]
  python -m paper_2605_26599_amd.profsum fp64 <counter.csv> <kernel_trace.csv> <bench.jsonl> <out.json> <out.md> <title> <command>

`stats` folds the per-instance kernel statistics of a `--kernel-trace --stats`
run into per-kernel totals and sets them beside the live HIP-event timing of
the same bench.py line.  `traffic` turns two `--pmc` runs (FETCH_SIZE, then
WRITE_SIZE; KiB per dispatch) into HBM bytes per launch for each kernel
family, scaled by the same counters' reading for a plain device copy of
known size (bench.py --calibrate-copy), and records the hash of the kernel
sources so bench.py reports the figure only while the kernels are unchanged;
with a kernel trace of the same configuration it also gives each family's
average duration and the HBM rate (bytes per launch over that duration)
against the 8 TB/s peak.
`fp64` sets hardware-counted FP64 FLOP/s (SQ_INSTS_VALU_*_F64 counters of a
`--pmc` run, durations from a `--kernel-trace` run of the same command) beside
the algorithmic FLOP/s of each kernel family.
"""
import csv
import json
import re
import sys
from collections import defaultdict


def _short(name: str) -> str:
    """Kernel name without namespaces, return type and parameter list."""
    name = name.replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", name).replace("void ", "").replace("tde::", "").strip()


def _family(name: str) -> str:
    return re.sub(r"<.*>", "", _short(name))


def stats(stats_csv, bench_jsonl, out_md, title, cmd):
    rows = list(csv.DictReader(open(stats_csv)))
    agg = {}
    for r in rows:
        a = agg.setdefault(_family(r["Name"]), [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
    tot = sum(v[1] for v in agg.values())
    lines = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", cmd, "```", "",
             "Per-kernel totals over the whole profiled run (all template instances of a kernel summed):", "",
             "| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {k} | {c} | {t / 1e6:.3f} | {t / c / 1e3:.2f} | {100 * t / tot:.1f}% |")
    lines += ["", "Instances as reported by rocprofv3 (`--stats`):", "",
              "| name | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
        short = _short(r["Name"])
        lines.append(f"| {short} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    b = json.loads([ln for ln in open(bench_jsonl) if ln.startswith("{")][-1])
    rf = b.get("roofline")
    if rf:
        # the eight-wave launches of wide-only levels belong to the same step, and
        # the in-wave whole-merge launches to the same kind as k_level_block
        fams = (rf["kernel"], rf["kernel"] + "_wide") + (("k_level_wave",) if rf["kernel"] == "k_level_block" else ())
        parts = [agg[k] for k in fams if k in agg]
        fam = [sum(p[0] for p in parts), sum(p[1] for p in parts)] if parts else None
        lines += ["", "The same workload as measured live by bench.py (HIP events, instrumented timed region):", "",
                  f"- ms per solve (un-instrumented timed region): {b['ms_per_step']:.3f}",
                  f"- dominant kernel: {rf['kernel']}, {rf['launches']} launches, "
                  f"average {rf['avg_launch_us']:.2f} us per launch",
                  (f"- rocprofv3 average for the same kernel family: {fam[1] / fam[0] / 1e3:.2f} us per launch"
                   if fam else "- (kernel family not in this trace)"),
                  f"- achieved {rf['achieved']:.4g} {rf['unit']} of {rf['peak']} "
                  f"({100 * rf['frac']:.2f}% of peak, bound: {rf['bound']})"]
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(path, counter):
    """Per-dispatch counter values (KiB) by kernel family."""
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", counter) != counter:
            continue
        vals[_family(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


PEAK_HBM_GBS = 8000.0


def traffic(fetch_csv, write_csv, copy_bytes, out_json, out_md, cmd, trace_csv=None):
    import os

    f = _counter(fetch_csv, "FETCH_SIZE")
    w = _counter(write_csv, "WRITE_SIZE")
    copy_bytes = float(copy_bytes)
    copy_names = [k for k in f if "copy" in k.lower() or "elementwise" in k.lower()]
    # the calibration copy is the largest-fetch copy dispatch
    best = max(((max(f[k]), k) for k in copy_names), default=None)
    if best is None:
        raise SystemExit("no copy kernel in the counter run")
    ck = best[1]
    kf = copy_bytes / (max(f[ck]) * 1024.0)
    kw = copy_bytes / (max(w[ck]) * 1024.0) if ck in w and max(w[ck]) > 0 else 1.0
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.dirname(here))
    import bench

    rec = {"calibration": {"kernel": ck, "copy_bytes": copy_bytes, "fetch_scale": kf, "write_scale": kw}}
    lines = ["# HBM traffic per launch (rocprofv3 hardware counters)", "", "Commands (repository root, one MI355X):",
             "", "```", cmd, "```", "",
             f"Calibration: one plain device copy of {copy_bytes / 2**20:.0f} MiB ({ck}); "
             f"scale factors fetch {kf:.4f}, write {kw:.4f} (known bytes / counter bytes).", ""]
    dur = defaultdict(list)
    if trace_csv:
        for fam, t in _dispatch_durations(trace_csv):
            dur[fam].append(t)
        lines += ["Durations: the average of each family's dispatches in a `--kernel-trace` run of the same "
                  "configuration; HBM rate = scaled bytes per launch / that average, against the 8 TB/s peak.", "",
                  "| kernel | dispatches | fetch KiB/launch (raw) | write KiB/launch (raw) | HBM bytes/launch (scaled) "
                  "| avg us | HBM GB/s | % of peak |", "|---|---|---|---|---|---|---|---|"]
    else:
        lines += ["| kernel | dispatches | fetch KiB/launch (raw) | write KiB/launch (raw) | HBM bytes/launch (scaled) |",
                  "|---|---|---|---|---|"]
    kinds = {"k_secular": "secular", "k_lowner": "lowner", "k_rows": "rows", "k_secular_wide": "secular",
             "k_lowner_wide": "lowner", "k_rows_wide": "rows", "k_leaf": "leaf", "k_leaf_dc": "leaf",
             "k_small_merge": "small", "k_level_block": "level", "k_merge": "merge", "k_assemble": "assemble"}
    for k in sorted(f, key=lambda k: -sum(f[k])):
        if k == ck:
            continue
        fm = sum(f[k]) / len(f[k])
        wm = (sum(w[k]) / len(w[k])) if k in w and w[k] else 0.0
        b = fm * 1024 * kf + wm * 1024 * kw
        row = f"| {k} | {len(f[k])} | {fm:.1f} | {wm:.1f} | {b:.4g} |"
        if trace_csv:
            if dur.get(k):
                us = sum(dur[k]) / len(dur[k]) / 1e3
                gbs = b / (us * 1e-6) / 1e9
                row += f" {us:.2f} | {gbs:.0f} | {100 * gbs / PEAK_HBM_GBS:.1f}% |"
            else:
                row += " | | |"
        lines.append(row)
        if k in kinds:
            rec[kinds[k]] = {"kernel": k, "bytes_per_launch": b, "source_hash": bench.source_hash()}
    json.dump(rec, open(out_json, "w"), indent=1)
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


# Kernel family -> bench.py launch kind (the kinds whose algorithmic work the
# library's counters measure).
KIND_OF = {"k_secular": "secular", "k_secular_wide": "secular", "k_lowner": "lowner", "k_lowner_wide": "lowner",
           "k_rows": "rows", "k_rows_wide": "rows", "k_small_merge": "small", "k_level_block": "level",
           "k_leaf": "leaf", "k_leaf_dc": "leaf"}
FP64_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64")
PEAK_FP64_TFLOPS = 78.6


def _dispatch_counters(path):
    """Per dispatch (in dispatch order): (family, {counter: value})."""
    by = {}
    for r in csv.DictReader(open(path)):
        did = int(r["Dispatch_Id"])
        ent = by.setdefault(did, [_family(r["Kernel_Name"]), {}])
        ent[1][r["Counter_Name"]] = ent[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [by[k] for k in sorted(by)]


def _dispatch_durations(path):
    """Per dispatch (in dispatch order): (family, duration ns)."""
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append((int(r["Dispatch_Id"]), _family(r["Kernel_Name"]),
                     int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    return [(f, t) for _, f, t in rows]


def fp64(counter_csv, trace_csv, bench_jsonl, out_json, out_md, title, cmd):
    """Hardware FP64 FLOP/s per kernel family: FLOPs from the SQ_INSTS_VALU_*_F64
    counters (64 lanes per wave instruction, an FMA counted as two), time from
    a kernel trace of the same command; the i-th dispatch of a family in one
    run is matched with the i-th in the other.  Beside it, the algorithmic
    rate from the library's work counters as bench.py accounts them."""
    import os

    cnt = _dispatch_counters(counter_csv)
    dur = _dispatch_durations(trace_csv)
    fl, tm = defaultdict(list), defaultdict(list)
    for f, c in cnt:
        fl[f].append(64.0 * (c.get(FP64_COUNTERS[0], 0.0) + c.get(FP64_COUNTERS[1], 0.0)
                             + c.get(FP64_COUNTERS[3], 0.0) + 2.0 * c.get(FP64_COUNTERS[2], 0.0)))
    for f, t in dur:
        tm[f].append(float(t))
    b = json.loads([ln for ln in open(bench_jsonl) if ln.startswith("{")][-1])
    work = b.get("work_flops_per_step", {})
    launches = b.get("launches_per_step_by_kind", {})
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.dirname(here))
    import bench

    lines = [f"# {title}", "", "Commands (repository root, one MI355X):", "", "```", cmd, "```", "",
             "Hardware FP64 FLOPs = 64 x (ADD_F64 + MUL_F64 + TRANS_F64 + 2 FMA_F64) wave instructions "
             "(`SQ_INSTS_VALU_*_F64`), over the kernel-trace durations of the same dispatches; peak "
             f"{PEAK_FP64_TFLOPS} TFLOP/s.  Algorithmic FLOPs are the library's work counters times bench.py's "
             "per-unit figures (6 per pole term, 3 per Loewner pair, 8 per row pair).", "",
             "| kernel | dispatches | HW GFLOP/launch | avg us | HW TFLOP/s | HW % of peak | algorithmic TFLOP/s "
             "| alg. % of peak |", "|---|---|---|---|---|---|---|---|"]
    rec = {"source_hash": bench.source_hash(), "kernels": {}}
    fams = [f for f in fl if f in tm and len(fl[f]) == len(tm[f])]
    for f in sorted(fams, key=lambda f: -sum(tm[f])):
        F, T = sum(fl[f]), sum(tm[f])
        if F <= 0 or T <= 0:
            continue
        hw = F / T / 1e3  # flop per ns = GFLOP/s; / 1e3 -> TFLOP/s
        kind = KIND_OF.get(f)
        alg = ""
        algp = ""
        if kind and kind in work and launches.get(kind):
            # every launch of the kind in the profiled run belongs to a solve
            # of the same workload: solves = dispatches of the kind / launches per solve
            kd = [g for g in fams if KIND_OF.get(g) == kind]
            solves = sum(len(tm[g]) for g in kd) / launches[kind]
            share = T / sum(sum(tm[g]) for g in kd)
            a = work[kind] * solves * share / T / 1e3
            alg, algp = f"{a:.3f}", f"{100 * a / PEAK_FP64_TFLOPS:.2f}%"
        n = len(fl[f])
        lines.append(f"| {f} | {n} | {F / n / 1e9:.4g} | {T / n / 1e3:.2f} | {hw:.3f} | "
                     f"{100 * hw / PEAK_FP64_TFLOPS:.2f}% | {alg} | {algp} |")
        rec["kernels"][f] = {"hw_flops_per_launch": F / n, "avg_us": T / n / 1e3, "hw_tflops": hw}
    # the largest dispatches of the widest kernel: the big merges of the solve
    for f in ("k_secular_wide", "k_secular"):
        if f in rec["kernels"] and len(tm[f]) > 0:
            order = sorted(range(len(tm[f])), key=lambda i: -tm[f][i])[:max(1, len(tm[f]) // 8)]
            F = sum(fl[f][i] for i in order)
            T = sum(tm[f][i] for i in order)
            lines += ["", f"Longest eighth of the `{f}` dispatches (the largest merges): {len(order)} dispatches, "
                          f"{T / len(order) / 1e3:.1f} us average, {F / T / 1e3:.3f} TFLOP/s hardware-counted "
                          f"({100 * F / T / 1e3 / PEAK_FP64_TFLOPS:.2f}% of peak)."]
            rec["kernels"][f]["hw_tflops_longest_eighth"] = F / T / 1e3
            break
    json.dump(rec, open(out_json, "w"), indent=1)
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:7])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:9])
    elif sys.argv[1] == "fp64":
        fp64(*sys.argv[2:9])
    else:
        raise SystemExit(__doc__)
