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


def test_profile_hash_follows_code_not_comments(tmp_path, monkeypatch):
    """A stored profile is reused while the kernels' and launchers' code is
    unchanged: editing a comment or the layout keeps the hash, editing code
    (here one launch constant of the host plan) changes it."""
    for f in bench.KERNEL_SOURCES:
        d = tmp_path / os.path.dirname(f)
        d.mkdir(parents=True, exist_ok=True)
        (tmp_path / f).write_text(open(os.path.join(bench.ROOT, f)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    k = tmp_path / bench.KERNEL_SOURCES[0]
    k.write_text("// a new comment line\n" + k.read_text().replace("\n{", "\n  {", 3))
    assert bench.kernel_source_hash() == h0
    a = tmp_path / "paper_1804_07135_amd/csrc/ssm_api.hip"
    src = a.read_text()
    assert "12288 / p.arc_chunks" in src
    a.write_text(src.replace("12288 / p.arc_chunks", "6144 / p.arc_chunks"))
    assert bench.kernel_source_hash() != h0


def test_replay_chunk_keeps_capture_out_of_the_timed_steps():
    """The warm-up builds the graph the timed steps replay: the chunk never
    exceeds the warm-up, and no warm-up means direct launches."""
    assert bench.replay_chunk(10, 10) == 10
    assert bench.replay_chunk(100, 10) == 10
    assert bench.replay_chunk(5, 10) == 5
    assert bench.replay_chunk(0, 10) == 0
    assert bench.replay_chunk(3, 0) == 0
