"""Host logic of bench.py that needs no GPU: the algorithmic byte model,
the kept-row fraction of the benchmark plate, the traffic-summary lookup
(source hash and kernel match), and the refusal of more than one GPU."""
import subprocess
import sys

import pytest

import bench
from paper_2102_11910_amd import workloads as wl


def test_kernel_bytes_match_the_convolution_model():
    n = 512
    kb = bench.kernel_bytes(n, 10000, 256, 2, True, 1.0)
    # one FP32 convolution: 44 n^2 to leading order (rows 12, cols 20, rows 12)
    conv32 = kb["rows_fwd"] - 8 * n * n + 4 * n * n + kb["cols"] + kb["rows_inv"]
    assert abs(conv32 / (44.0 * n * n) - 1.0) < 0.02
    # the FP64 column pass reads and writes complex doubles and a real FP64 spectrum
    assert kb["cols64"] == 32 * n * (n + 1) + 8 * (n + 1) ** 2


def test_kept_rows_of_the_benchmark_plate():
    keep = bench.kept_rows(wl.config2())
    # the 20 degree plate spans about 70 rows; whole 16-row groups: 96 of 512
    assert keep == 96 / 512


def test_traffic_lookup_checks_source_and_kernel(tmp_path, monkeypatch):
    src = bench.source_hash("fft_conv.hip")
    f = tmp_path / "traffic.md"
    f.write_text(
        f"class cols64: fetch_bytes=100 write_bytes=20 source=fft_conv.hip@{src} kernels=1 "
        "matched=k_cols_conv_split<double\n"
        f"class rows_fwd: fetch_bytes=7 write_bytes=3 source=fft_conv.hip@{src} kernels=1 "
        "matched=k_rows_fwd<double,float\n"
        "class cols: fetch_bytes=1 write_bytes=1 source=fft_conv.hip@0000 kernels=1 "
        "matched=k_cols_conv<float\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(f))
    assert bench.measured_traffic("cols64", "k_cols_conv_split<double") == 120.0
    assert bench.measured_traffic("cols64") == 120.0
    assert bench.measured_traffic("cols64", "k_cols_conv<double") is None   # another kernel
    assert bench.measured_traffic("rows_fwd", "k_rows_fwd<double, float") == 10.0
    assert bench.measured_traffic("cols") is None                            # stale source
    assert bench.measured_traffic("velocity") is None                        # not measured


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_problem_bytes_of_the_merged_batch():
    """Per problem of the merged batch: two FP32 convolutions (the first
    keeping a band of rows) to 88 n^2 at full band, or the FP64 first
    convolution in its own classes."""
    n, band = 1024, 1024
    pb = bench.problem_bytes(n, 5000, 300, 0, False, band)
    conv = pb["rows_fwd"] + pb["cols"] + pb["rows_inv"]
    assert abs(conv / (88.0 * n * n) - 1.0) < 0.02
    assert pb["scatter"] == 24 * 5000 + 4 * n * n
    p64 = bench.problem_bytes(n, 5000, 300, 0, True, 96)
    assert "cols64" in p64 and p64["rows_fwd"] == 8 * n * n + 8 * n * (n + 1)
    assert p64["cols64"] == 16 * n * (n + 1) + 8 * (n + 1) ** 2 + 16 * (n + 1) * 96


def test_trace_and_counter_summaries(tmp_path, monkeypatch):
    """The profile summarizers read rocprofv3's CSV layout and write one row
    per kernel class and per kernel."""
    import csv
    import json
    td = tmp_path / "trace" / "host"
    td.mkdir(parents=True)
    names = ["void gpf::(anonymous namespace)::k_cols_multi<float>(gpf::ConvDesc const*, gpf::MultiPass)",
             "gpf::(anonymous namespace)::k_bin_count(gpf::ProbDesc const*, gpf::FlatMap)"]
    with open(td / "c4_kernel_stats.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"])
        w.writerow([names[0], 135, 135 * 97000, 97000, 60.0, 90000, 110000])
        w.writerow([names[1], 90, 90 * 20000, 20000, 40.0, 1000, 50000])
    # the trace: 5 warmup steps, 20 event-timed steps, 20 headline steps; per
    # step 3 column dispatches (100, 97, 110 us in the three phases) and 2
    # bin counts of 20 us; the per-class rows use the event-timed steps only
    with open(td / "c4_kernel_trace.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 1000
        for step in range(45):
            cols_ns = 100000 if step < 5 else (97000 if step < 25 else 110000)
            for nm, dur, k in ((names[1], 20000, 2), (names[0], cols_ns, 3)):
                for _ in range(k):
                    w.writerow([nm, t, t + dur])
                    t += dur + 500
    res = {"warmup": 5, "steps": 20, "ms_per_step": 1.2,
           "roofline": {"kernel": "cols", "avg_us": 97.5, "achieved": 2900.0, "frac": 0.36},
           "kernels": {"cols": {"us_per_step": 292.0, "avg_us": 97.5}}}
    bj = tmp_path / "bench.json"
    bj.write_text("[bench] log line\n" + json.dumps(res) + "\n")
    out = tmp_path / "trace.md"
    monkeypatch.setattr(bench, "TRACE_SUMMARY", str(out))
    bench.summarize_trace(str(tmp_path / "trace"), str(bj))
    text = out.read_text()
    # the 60 column dispatches of the event-timed steps, 97 us each: 3 per
    # step, 291 us per step
    assert "| cols | 1 | 291.00 | 97.00 | 3.00 | 292.00 | 97.50 |" in text
    assert "| scatter | 1 | 40.00 | 20.00 | 2.00 |" in text
    assert "| k_bin_count | 90 | 20.00 |" in text

    sq = []
    for i, counters in enumerate((("SQ_WAVES", "SQ_INSTS_VALU"), ("SQ_WAVES", "SQ_BUSY_CYCLES"))):
        d = tmp_path / f"sq{i}" / "host"
        d.mkdir(parents=True)
        with open(d / "pmc_counter_collection.csv", "w", newline="") as fh:
            w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for disp in range(2):
                for c in counters:
                    v = {"SQ_WAVES": 100.0, "SQ_INSTS_VALU": 5000.0 * (disp + 1), "SQ_BUSY_CYCLES": 7.0}[c]
                    w.writerow({"Dispatch_Id": disp, "Kernel_Name": names[0], "Counter_Name": c,
                                "Counter_Value": v})
        sq.append(str(tmp_path / f"sq{i}"))
    out = tmp_path / "sq.md"
    monkeypatch.setattr(bench, "SQ_SUMMARY", str(out))
    bench.summarize_sq(sq)
    text = out.read_text()
    assert "--pmc SQ_INSTS_VALU SQ_WAVES" in text and "--pmc SQ_BUSY_CYCLES SQ_WAVES" in text
    assert "| k_cols_multi<float> | 2 | 100 | 75 |" in text
