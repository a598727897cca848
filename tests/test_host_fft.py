"""The LDS FFT passes of the HIP kernels, run on the host with the 64 lanes
of a wavefront emulated in lockstep, against a naive long-double DFT (all
lengths 1..1024, FP32 and FP64, forward and inverse, every radix cap, for the
runtime-length passes and the compile-time-length ones)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fft_passes_on_host(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "fft_host_check"
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_1804_07135_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "fft_host_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:]
    assert out.stdout.strip().endswith("OK")
