"""Host-side tools, no GPU: the benchmark's single-GPU guard and the
rocprofv3 summarisers that fill profiles/ (kernel families folded across
template instances, counter scaling by the calibration copy, the source hash
that invalidates stale traffic figures)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_profsum_stats_folds_instances(tmp_path):
    from paper_2605_26599_amd import profsum

    stats = tmp_path / "stats.csv"
    _write(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"], [
        ["void tde::k_small_merge<1024>(tde::MergeRec const*)", 4, 400000, 100000, 90000, 110000],
        ["void tde::k_small_merge<512>(tde::MergeRec const*)", 1, 50000, 50000, 50000, 50000],
        ["void tde::k_secular_wide<8>(tde::MergeRec const*)", 2, 20000, 10000, 9000, 11000],
        ["void tde::k_secular<16>(tde::MergeRec const*)", 2, 20000, 10000, 9000, 11000],
    ])
    bench_out = tmp_path / "bench.txt"
    line = {"ms_per_step": 1.0, "roofline": {"kernel": "k_secular", "launches": 4, "avg_launch_us": 10.0,
                                              "achieved": 1.0, "unit": "TFLOP/s", "peak": 78.6, "frac": 0.0127,
                                              "bound": "alu"}}
    bench_out.write_text("noise\n" + json.dumps(line) + "\n")
    md = tmp_path / "out.md"
    profsum.stats(str(stats), str(bench_out), str(md), "title", "the command")
    text = md.read_text()
    # both template instances of the fused kernel in one row: 5 calls, 0.450 ms
    assert "| k_small_merge | 5 | 0.450 | 90.00 |" in text
    # the eight-wave launches count with the step they belong to: 4 calls, 40 us total
    assert "rocprofv3 average for the same kernel family: 10.00 us per launch" in text
    assert "the command" in text


def test_profsum_traffic_scales_by_the_copy(tmp_path):
    import bench
    from paper_2605_26599_amd import profsum

    copy_bytes = 256 * 2**20
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the counters read half the copy's fetched bytes and all of its written bytes
    _write(fetch, hdr, [["__amd_rocclr_copyBuffer", "FETCH_SIZE", copy_bytes / 2048],
                        ["void tde::k_small_merge<1024>(x)", "FETCH_SIZE", 100.0],
                        ["void tde::k_small_merge<1024>(x)", "FETCH_SIZE", 300.0]])
    _write(write, hdr, [["__amd_rocclr_copyBuffer", "WRITE_SIZE", copy_bytes / 1024],
                        ["void tde::k_small_merge<1024>(x)", "WRITE_SIZE", 50.0],
                        ["void tde::k_small_merge<1024>(x)", "WRITE_SIZE", 50.0]])
    js, md = tmp_path / "t.json", tmp_path / "t.md"
    profsum.traffic(str(fetch), str(write), str(copy_bytes), str(js), str(md), "cmd")
    rec = json.loads(js.read_text())
    assert rec["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["calibration"]["write_scale"] == pytest.approx(1.0)
    # mean fetch 200 KiB x 2 + mean write 50 KiB x 1
    assert rec["small"]["bytes_per_launch"] == pytest.approx((200 * 2 + 50) * 1024)
    assert rec["small"]["source_hash"] == bench.source_hash()


def test_committed_traffic_record_names_known_kernels():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert rec["calibration"]["fetch_scale"] > 0 and rec["calibration"]["write_scale"] > 0
    for kind, r in rec.items():
        if kind == "calibration":
            continue
        assert r["kernel"].startswith("k_") and r["bytes_per_launch"] > 0 and len(r["source_hash"]) == 16


def test_profsum_fp64_counts_lanes_and_fma(tmp_path):
    """Hardware FLOPs = 64 lanes x (ADD + MUL + TRANS + 2 FMA) wave
    instructions per dispatch, over the kernel-trace durations of the same
    dispatches (matched in order); the algorithmic rate uses bench.py's work
    per solve and launches per solve."""
    from paper_2605_26599_amd import profsum

    cnt, trace = tmp_path / "c.csv", tmp_path / "t.csv"
    rows = []
    for did in (1, 2):
        for c, v in [("SQ_INSTS_VALU_ADD_F64", 100.0), ("SQ_INSTS_VALU_MUL_F64", 10.0),
                     ("SQ_INSTS_VALU_FMA_F64", 50.0), ("SQ_INSTS_VALU_TRANS_F64", 5.0)]:
            rows.append([did, "void tde::k_secular_wide<8>(x)", c, v])
    _write(cnt, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    _write(trace, ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [[1, "void tde::k_secular_wide<8>(x)", 1000, 2000], [2, "void tde::k_secular_wide<8>(x)", 5000, 8000]])
    bench_out = tmp_path / "b.txt"
    bench_out.write_text(json.dumps({"work_flops_per_step": {"secular": 4.0e5},
                                     "launches_per_step_by_kind": {"secular": 1}}) + "\n")
    js, md = tmp_path / "f.json", tmp_path / "f.md"
    profsum.fp64(str(cnt), str(trace), str(bench_out), str(js), str(md), "title", "cmd")
    rec = json.loads(js.read_text())["kernels"]["k_secular_wide"]
    per = 64 * (100 + 10 + 5 + 2 * 50)
    assert rec["hw_flops_per_launch"] == pytest.approx(per)
    # 2 launches, 4000 ns in all: flop/ns = GFLOP/s, / 1e3 = TFLOP/s
    assert rec["hw_tflops"] == pytest.approx(2 * per / 4000 / 1e3)
    # two solves of 4e5 algorithmic flops over 4000 ns
    assert "| 0.200 |" in md.read_text()
