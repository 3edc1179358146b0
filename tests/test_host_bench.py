"""Host logic of bench.py (CPU): the roofline entry computed from the
library's per-kernel profile (algorithmic bytes or matrix-core flops per
launch over the mean launch time, against MI355X's published peaks), the
per-step kernel table of the fully profiled steps, and the refusal of more
than one GPU before anything touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_hbm_roofline_of_a_kernel():
    # 10 launches of 805.3 MB in 1.453 ms in all -> 5542 GB/s of 8000
    d = {"launches": 10, "ms": 1.453, "bytes": 10 * 805.3e6}
    r = bench.kernel_roofline("smooth_color", d)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(805.3e6 / 0.1453e-3 / 1e9, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-12)
    assert r["avg_launch_ms"] == pytest.approx(0.1453, rel=1e-12)
    assert r["traffic"] is None


def test_mfma_roofline_of_the_net():
    # 5 layers of 13,824 flop per voxel on 512^3 voxels in 4 ms each
    per = 13824.0 * 512**3
    d = {"launches": 5, "ms": 20.0, "bytes": 5 * per}
    r = bench.kernel_roofline("conv3d_mfma", d)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 2500.0
    assert r["achieved"] == pytest.approx(per / 4e-3 / 1e12, rel=1e-12)


def test_roofline_entry_and_kernel_table():
    per = 10.0 * 512**3                 # fused sweeps: 10 bytes per cell
    timed = {"sweep4_fused": {"launches": 240, "ms": 112.6, "bytes": 240 * per}}
    full = {"sweep4_fused": {"launches": 36, "ms": 16.9, "bytes": 36 * per},
            "rhs": {"launches": 6, "ms": 5.8, "bytes": 6 * 3.22e9},
            "unused": {"launches": 0, "ms": 0.0, "bytes": 0.0}}
    r = bench.roofline_of(timed, full, 3)
    assert r["kernel"] == bench.ROOFLINE_KERNEL == "sweep4_fused"
    assert r["launches"] == 240
    assert r["achieved"] == pytest.approx(per / (112.6e-3 / 240) / 1e9, rel=1e-12)
    assert r["largest_kernel_in_full_profile"] == "sweep4_fused"
    assert set(r["kernels"]) == {"sweep4_fused", "rhs"}          # unused kernels left out
    assert r["kernels"]["rhs"]["ms_per_step"] == pytest.approx(5.8 / 3, abs=1e-3)
    assert r["kernels"]["rhs"]["launches_per_step"] == 2.0
    assert r["kernels"]["rhs"]["GB/s"] == pytest.approx(6 * 3.22e9 / 5.8e-3 / 1e9, abs=0.1)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout == ""


def test_net_flops_per_voxel():
    # method: 3 -> 16, 16 -> 16 (x3), 16 -> 1 channels of 3^3 taps, 2 flop per tap
    assert bench.NET_METHOD_FLOPS_PER_VOXEL == 2 * 27 * (48 + 768 + 16) == 44928
    # kernels: every layer padded to 16 x 16 channels
    assert bench.NET_KERNEL_FLOPS_PER_VOXEL == 5 * 13824 == 69120


def test_measured_traffic_matches_the_committed_counters():
    # the HBM bytes per launch the bench line carries for its roofline kernel
    # are the committed rocprofv3 summary's figures for the 512^3 level's
    # post-smoothing pass: FETCH_SIZE scaled by the copy probe, plus WRITE_SIZE
    import re
    path = os.path.join(ROOT, "profiles", "pm_step_512_mixed_hbm_traffic.md")
    text = open(path).read()
    probe = re.search(r"dispatch 2\): FETCH_SIZE ([0-9.]+) KiB", text)
    row = re.search(r"^\| k_sweep4<false, false, false, 16, 32, 768> \| \d+ \| \d+ \| ([0-9.]+) \| ([0-9.]+) \|",
                    text, re.M)
    assert probe and row
    fetch, write = float(row.group(1)), float(row.group(2))
    total = fetch * 1024 * 1048576 / float(probe.group(1)) + write * 1024
    assert bench.MEASURED_TRAFFIC["sweep4_fused"] == pytest.approx(total, rel=1e-6)
