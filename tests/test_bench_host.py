"""Host logic of the benchmark and the binding: the algorithmic byte and
flop counts the roofline uses (checked against hand-computed values for the
256x256x8, 48-image workload), the one-GPU refusal, and the binding failing
loudly when the HIP library is absent (no fallback path)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1804_07135_amd import inputs  # noqa: E402

TUBE = inputs.WORKLOADS["tube_256x256x8_k48"]


def test_algorithmic_bytes_of_the_tube_workload():
    ab = bench.algorithmic_bytes(TUBE, 4)
    spins = 48 * 3 * 256 * 256 * 8 * 4             # one FP32 string
    xspec = 48 * 257 * 3 * 8 * 256 * 2 * 4          # x half-spectra: (m_x + 1) = 257 columns, complex
    nhat = 257 * 512 * 16 * 6 * 4                   # six real kernel components on the half grid
    assert ab["k_xfwd"] == spins + xspec
    assert ab["k_conv"] == 2 * xspec + nhat == 1263206400
    assert ab["k_xinv"] == xspec + 2 * spins
    assert ab["k_arc"] == spins
    # interpolation: every source image read once (consecutive targets
    # share their sources) and every image written once
    assert ab["k_interp"] == 2 * spins


def test_roofline_is_hbm_with_executed_flop_alu_view():
    """The headline roofline is the HBM one (algorithmic bytes over the
    launch time against 8 TB/s); the vector-ALU view uses executed flops
    from the counters against the non-packed FP32 ceiling (256 CUs x 4 SIMDs
    x 16 lanes x 2 flops x 2.4 GHz)."""
    assert bench.HBM_PEAK_GBS == 8000.0
    assert abs(bench.FP32_VECTOR_NONPACKED_TFLOPS - 256 * 4 * 16 * 2 * 2.4e9 / 1e12) < 0.05
    assert not hasattr(bench, "conv_algorithmic_flops")


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_binding_fails_loudly_without_the_library(tmp_path):
    code = ("import paper_1804_07135_amd.ssm as s\n"
            f"s.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
            "s._lib = None\n"
            "try:\n"
            "    s.ssm_version()\n"
            "except RuntimeError as e:\n"
            "    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert "raised" in r.stdout and "missing" in r.stdout
