"""Host logic of bench.py (no GPU): the one-GPU refusal, the slice-product operation count, and the
roofline record built from per-kind launch timing."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KINDS = ("gemm", "dd_gemm", "oz_gemm")


def _prof(**ms_flops):
    p = {k: {"launches": 0, "ms": 0.0, "flops": 0.0} for k in KINDS + ("gather",)}
    for k, (launches, ms, flops) in ms_flops.items():
        p[k] = {"launches": launches, "ms": ms, "flops": flops}
    return p


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_int8_operations_per_complex_multiply_add():
    # slice pairs s + t <= S - 1 of S slices, three real products (Gauss), two operations per multiply-add
    assert bench.oz_int8_ops_per_cmac(16) == 3 * 136 * 2 == 816
    assert bench.oz_int8_ops_per_cmac(15) == 3 * 120 * 2
    assert bench.oz_int8_ops_per_cmac(0) == 816


def test_roofline_of_the_slice_product():
    # 10 launches of 4.7e10 flops in 25 ms: 18.8 TFLOP/s
    prof = _prof(oz_gemm=(10, 25.0, 4.7e11), dd_gemm=(5, 3.0, 1e10), gather=(3, 2.0, 0.0))
    r = bench.roofline_of(prof, 3, {"oz_gemm": 10 * 3.2e9}, 16)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(18.8)
    assert r["frac"] == pytest.approx(18.8 / bench.FP64_MFMA_PEAK_TFLOPS)
    assert r["avg_launch_ms"] == pytest.approx(2.5) and r["launches"] == 10
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(3.2e9)
    assert r["share_of_kernel_time"] == pytest.approx(25.0 / 30.0)
    assert r["int8_matrix_cores"]["achieved"] == pytest.approx(18.8 * 816 / 8)
    # traffic comes from counters taken with 16 slices only
    assert bench.roofline_of(prof, 3, None, 15)["traffic"] is None


def test_roofline_of_the_vector_and_fp64_paths():
    r = bench.roofline_of(_prof(dd_gemm=(4, 10.0, 4e10), gemm=(2, 1.0, 1e9)), 2)
    assert r["bound"] == "alu" and r["achieved"] == pytest.approx(4.0)
    r0 = bench.roofline_of(_prof(gemm=(8, 4.0, 1.6e11)), 0)
    assert r0["bound"] == "mfma" and r0["achieved"] == pytest.approx(40.0) and r0["avg_launch_ms"] == 0.5


def test_traffic_hash_covers_existing_sources():
    h = bench.oz_sources_sha256()
    assert h is not None and re.fullmatch(r"[0-9a-f]{64}", h)
