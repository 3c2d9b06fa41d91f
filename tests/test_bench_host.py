"""Host-side pieces of bench.py: the algorithmic byte counts it divides by,
the hardware-counter summary it builds from rocprofv3 output, and its
one-GPU guard.  No GPU is used."""
import csv
import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_pipeline_bytes_counts_each_kernel_once():
    W, H, Dp, P = 4, 2, 64, 4
    px, N = W * H, W * H * Dp
    # census: 2 images in, 2 u64 maps out; cost: 2 maps in, N out;
    # aggregation: N in and N out per direction; WTA: P planes in, 2 u16 maps out
    expect = (2 * px + 16 * px) + (16 * px + N) + 2 * P * N + (P * N + 4 * px)
    assert bench.pipeline_bytes(W, H, Dp, P, (32, 16, 0, 0)) == expect == (3 * P + 1) * N + 38 * px
    # the headline workload
    assert bench.pipeline_bytes(640, 480, 128, 4, (32, 16, 0, 0)) == 522_854_400


def test_pipeline_bytes_of_the_fused_variants():
    W, H, Dp, P = 8, 3, 128, 8
    px, N = W * H, W * H * Dp
    fused = (2 * px + 16 * px) + P * (16 * px + N) + (P * N + 4 * px)
    assert bench.pipeline_bytes(W, H, Dp, P, (32, 16, 1, 0)) == fused
    census_cost = (2 * px + N) + 2 * P * N + (P * N + 4 * px)
    assert bench.pipeline_bytes(W, H, Dp, P, (32, 16, 0, 1)) == census_cost


def test_pipeline_bytes_with_the_final_pass():
    # the last direction's plane is neither written nor read: 2N fewer bytes
    W, H, Dp = 8, 3, 128
    px, N = W * H, W * H * Dp
    for P in (2, 4, 8):
        plain = bench.pipeline_bytes(W, H, Dp, P, (32, 16, 0, 0, 0))
        fp = bench.pipeline_bytes(W, H, Dp, P, (32, 16, 0, 0, 1))
        assert plain - fp == 2 * N
        assert fp == (2 * px + 16 * px) + (16 * px + N) + 2 * (P - 1) * N + (N + (P - 1) * N + 4 * px)
        assert bench.pipeline_bytes(W, H, Dp, P, (32, 16, 0, 1, 1)) == \
            bench.pipeline_bytes(W, H, Dp, P, (32, 16, 0, 1, 0)) - 2 * N
    # the final pass needs the stored cost volume: ignored with fused costs
    assert bench.pipeline_bytes(W, H, Dp, 4, (32, 16, 1, 0, 1)) == bench.pipeline_bytes(W, H, Dp, 4, (32, 16, 1, 0))


def _write_pmc(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_summary_scales_by_the_copy(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    agg = "void sgm::aggregate_kernel<32, 16, 128, unsigned char, false, false>(sgm::AggArgs)"
    cost = "void sgm::cost_kernel<false>(sgm::CostArgs)"
    mib = 256
    # FETCH_SIZE reads half of a copy's bytes, WRITE_SIZE all of them; small
    # copies (image uploads) in the same run do not enter the calibration
    _write_pmc(tmp_path / "f.csv", "FETCH_SIZE",
               [(copy, mib * 512.0), (copy, 1.5), (copy, mib * 512.0), (agg, 1000.0), (agg, 1002.0), (cost, 10.0)])
    _write_pmc(tmp_path / "w.csv", "WRITE_SIZE",
               [(copy, mib * 1024.0), (copy, 0.03), (agg, 3000.0), (cost, 20.0)])
    s = bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), mib, ["32", "16", "0", "0"])
    assert s["kernel"] == agg and s["tuning"] == [32, 16, 0, 0]
    assert s["fetch_scale"] == 2.0 and s["write_scale"] == 1.0
    assert s["bytes_per_launch"] == 1001.0 * 2 * 1024 + 3000.0 * 1024
    assert s["kernels"][cost]["read_bytes"] == 20 * 1024
    assert copy not in s["kernels"]
    assert "fetch_scale_read_only" not in s
    json.dumps(s)
    # with the read-only reduction of the same size: its scale is reported
    red = "void at::native::reduce_kernel<512, 1>"
    _write_pmc(tmp_path / "f2.csv", "FETCH_SIZE",
               [(copy, mib * 512.0), (red, mib * 512.0 * 1.0005), (agg, 1000.0)])
    _write_pmc(tmp_path / "w2.csv", "WRITE_SIZE", [(copy, mib * 1024.0), (red, 16.0), (agg, 3000.0)])
    s2 = bench.summarize_counters(str(tmp_path / "f2.csv"), str(tmp_path / "w2.csv"), mib, ["32", "16", "0", "0"])
    assert abs(s2["fetch_scale_read_only"] - 2.0) < 0.01
    assert red not in s2["kernels"]


@pytest.mark.parametrize("n", [0, 2, 8])
def test_bench_runs_on_one_gpu_only(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    a = tmp_path / "a.h"
    a.write_text("int f(int x) {  // one\n    return x + 1; /* two */\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SRCS", [str(a)])
    h0 = bench._kernel_sha()
    a.write_text("int f(int x) {\n  // another comment\n  return x + 1;\n}\n")
    assert bench._kernel_sha() == h0
    a.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench._kernel_sha() != h0


def test_committed_traffic_summary_is_used_only_for_the_kernels_it_measured():
    # bench.py reports the committed byte counters only while the kernels are
    # the ones they were taken from (same source hash and kernel shape);
    # otherwise traffic is null
    summary = json.load(open(bench.TRAFFIC_FILE))
    if summary["kernel_sha"] == bench._kernel_sha():
        assert bench._traffic(tuple(summary["tuning"])) == summary["bytes_per_launch"]
    else:
        assert bench._traffic(tuple(summary["tuning"])) is None
    other = list(summary["tuning"])
    other[0] = 16 if other[0] != 16 else 32
    assert bench._traffic(tuple(other)) is None
    # the context reports a longer tuning tuple (final pass, post stage inside
    # the WTA): those switches off is the counted shape, either on is not
    if summary["kernel_sha"] == bench._kernel_sha():
        assert bench._traffic(tuple(summary["tuning"]) + (False, False)) == summary["bytes_per_launch"]
    assert bench._traffic(tuple(summary["tuning"]) + (True, False)) is None
    assert bench._traffic(tuple(summary["tuning"]) + (False, True)) is None
    # every L_r byte written once; reads at most the algorithmic ones (L2 hits
    # may serve part of a slice's second read), so no wasted re-reads
    agg = summary["kernels"][summary["kernel"]]
    alg_half = 4 * 640 * 480 * 128
    assert abs(agg["write_bytes"] - alg_half) < 0.01 * alg_half
    assert 0.5 * alg_half < agg["read_bytes"] < 1.1 * alg_half


def test_bench_rejects_an_unknown_workload():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "no_such_workload"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "unknown workload" in r.stderr


def test_trace_summary_frames_and_gaps(tmp_path):
    """Frames start at each census launch; spans, kernel time and the gaps
    before each kernel and between frames come from the timestamps."""
    hdr = '"Kind","Kernel_Name","Start_Timestamp","End_Timestamp"\n'
    rows, t = [], 0
    for f in range(10):
        for name, dur, gap in (("sgm::(anonymous namespace)::census97_kernel(sgm::dev::CensusArgs)", 5000, 0),
                               ("void sgm::(anonymous namespace)::cost_kernel<false, 128>(sgm::dev::CostArgs)", 10000, 1000),
                               ("void sgm::(anonymous namespace)::wta_kernel<unsigned char, false>(sgm::dev::WtaArgs)",
                                20000, 2000)):
            t += gap
            rows.append(f'"KERNEL_DISPATCH","{name}",{t},{t + dur}\n')
            t += dur
        t += 8000  # between frames
    p = tmp_path / "t_kernel_trace.csv"
    p.write_text(hdr + "".join(rows))
    s = bench.summarize_trace(str(p), skip_frac=0.0)
    assert s["frames"] == 10 and s["kernels_per_frame"] == 3
    assert s["span_us"] == 38.0 and s["kernel_time_us"] == 35.0 and s["idle_in_frame_us"] == 3.0
    assert s["gap_us"] == {"census97_kernel -> cost_kernel": 1.0, "cost_kernel -> wta_kernel": 2.0}
    assert s["gap_between_frames_us"] == 8.0
