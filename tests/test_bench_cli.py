"""Host-side checks of the benchmark's command line (no GPU work): more than
one GPU is refused with a message, and the per-unit constants behind the
roofline entries are the documented products."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_constants():
    sys.path.insert(0, ROOT)
    import bench

    # contact tests of the structure kernel: M (M - 1) / 2 lipid pairs x 4 tail pairs x 15 ops
    assert bench.structure_ops_per_config(125) == 7750 * 4 * 15
    # Potts attempt: 205 VALU issue slots per lane; peak 256 CU x 64 lanes x 2.4 GHz (no packed fp32)
    assert bench.ALU_SLOTS_PER_ATTEMPT == 138 + 11 + 12 + 16 + 3 + 21 + 4 == 205
    assert abs(bench.VALU_LANE_SLOTS_PEAK - 3.93216e13) < 1e8
    assert abs(bench.FP64_UNFUSED_PEAK_TFLOPS - 39.3216) < 1e-6
    assert abs(bench.LDS_PEAK_GBS - 78643.2) < 1e-6
    r = bench.potts_roofline(640_000, 1.812, 20, None)
    assert abs(r["frac"] - 205 * 640_000 / 1.812e-3 / 3.93216e13) < 1e-12
    assert abs(r["lds"]["frac"] - 38 * 640_000 / 1.812e-3 / 78.6432e12) < 1e-12
    rb = bench.batched_roofline(8.96e9, 0.6735)
    assert abs(rb["frac"] - 205 * 8.96e9 / 0.6735 / 3.93216e13) < 1e-12
    assert abs(rb["lds"]["frac"] - 38 * 8.96e9 / 0.6735 / 78.6432e12) < 1e-12
    # HBM bytes: FETCH_SIZE x 2 + WRITE_SIZE x 1, in KiB, as recorded with the profiles
    assert abs(bench.STRUCT_4096_HBM_BYTES - (12588.7 * 2 + 256.0) * 1024) < 1000
    assert abs(bench.LIPID_SWEEP_HBM_BYTES - (792.67 * 2 + 1302.0) * 1024) < 1000
    assert abs(bench.TRIMER_SWEEP_HBM_BYTES - (227.75 * 2 + 308.0) * 1024) < 1000
    assert abs(bench.K_SWEEP_L32_HBM_BYTES - (268.18 * 2 + 390.0) * 1024) < 1000


def test_host_cpu_info():
    sys.path.insert(0, ROOT)
    import bench

    hc = bench.host_cpu()
    assert hc["usable"] >= 1 and hc["usable"] <= hc["affinity"] <= (os.cpu_count() or 1)
    threads, _ = bench.oracle_threads(3)
    assert 1 <= threads <= 3


def test_trace_window_averages_the_timed_launches(tmp_path):
    # a synthetic rocprofv3 csv trace: k_sweep dispatch i lasts 1000 + i ns,
    # a k_sync of 100 ns after each; the timed window is launches [5, 15)
    import csv
    import json

    sys.path.insert(0, ROOT)
    import bench

    (tmp_path / "host").mkdir()
    rows, t = [("Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp")], 0
    for i in range(20):
        rows.append((2 * i, "void rewl_gpu::(anonymous namespace)::k_sweep<0>(rewl_gpu::DevState, long, long)",
                     t, t + 1000 + i))
        t += 2000
        rows.append((2 * i + 1, "void rewl_gpu::(anonymous namespace)::k_sync<0>(rewl_gpu::DevState, long)",
                     t, t + 100))
        t += 200
    with open(tmp_path / "host" / "p_kernel_trace.csv", "w", newline="") as f:
        csv.writer(f).writerows(rows)
    line = {"config": {"timed_k_sweep_launches": [5, 15]}, "roofline": {"kernel_avg_ms": 1e-3}, "value": 1.0}
    (tmp_path / "b.json").write_text("[bench] log line\n" + json.dumps(line) + "\n")
    r = bench.trace_window(str(tmp_path), str(tmp_path / "b.json"))
    assert r["window_n"] == 10 and r["k_sweep_dispatches"] == 20
    assert abs(r["window_avg_ms"] - (1000 + 9.5) * 1e-6) < 1e-12
    assert r["window_min_ms"] == 1005e-6 and r["window_max_ms"] == 1014e-6
    o = r["other_kernels_in_window"]
    assert list(o) == ["k_sync<0>"] and o["k_sync<0>"]["n"] == 9 and abs(o["k_sync<0>"]["avg_ms"] - 1e-4) < 1e-15


def test_phase_clock_summary_per_attempt_and_per_block():
    # two walkers' counters in the order of the binding's PHASE_CLOCK_FIELDS
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import paper_1312_3004_amd as pk

    f = pk.PHASE_CLOCK_FIELDS
    assert len(f) == 12 and f[:8] == ("lane_cycles", "decide_cycles", "segments", "rounds", "exact_attempts",
                                      "blocks", "round_cycles", "attempts")
    row = dict(lane_cycles=700, decide_cycles=8000, segments=11, rounds=30, exact_attempts=1, blocks=10,
               round_cycles=3600, attempts=640, setup_cycles=640, commit_cycles=1280, exact_cycles=64,
               tail_cycles=320)
    ctr = np.array([[row[k] for k in f], [2 * row[k] for k in f]], dtype=np.uint64)
    s = bench.phase_clock_summary(ctr, f)
    assert s["attempts"] == 3 * 640
    assert abs(s["lane_parallel_cycles_per_attempt"]["mean"] - 700 / 640) < 1e-12
    assert abs(s["decision_cycles_per_attempt"]["max"] - 8000 / 640) < 1e-12
    assert abs(s["segments_per_block"]["mean"] - 1.1) < 1e-12
    assert abs(s["rounds_per_segment"] - 90 / 33) < 1e-12
    assert abs(s["commit_cycles_per_attempt"]["mean"] - 2.0) < 1e-12
    assert abs(s["exact_attempts_per_block"]["mean"] - 0.1) < 1e-12
