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
    # HBM bytes: FETCH_SIZE x 2 + WRITE_SIZE x 1, in KiB, as recorded with the profiles
    assert abs(bench.STRUCT_4096_HBM_BYTES - (12588.7 * 2 + 256.0) * 1024) < 1000
    assert abs(bench.LIPID_SWEEP_HBM_BYTES - (907.06 * 2 + 1302.0) * 1024) < 1000
    assert abs(bench.TRIMER_SWEEP_HBM_BYTES - (242.5 * 2 + 308.0) * 1024) < 1000
    assert abs(bench.K_SWEEP_L32_HBM_BYTES - (282.10 * 2 + 390.0) * 1024) < 1000


def test_host_cpu_info():
    sys.path.insert(0, ROOT)
    import bench

    hc = bench.host_cpu()
    assert hc["usable"] >= 1 and hc["usable"] <= hc["affinity"] <= (os.cpu_count() or 1)
    threads, _ = bench.oracle_threads(3)
    assert 1 <= threads <= 3
