"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code:
the oracle (gcc) driven through every entry point (tests/host/
oracle_sanitize.c), and the library's host side (batch planner, argument
checks, error reporting; host code only is instrumented, the GPU code is
built as usual) driven without a GPU (tests/host/plan_sanitize.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", str(exe),
                           os.path.join(ROOT, "tests", "host", "oracle_sanitize.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), (r.stdout + r.stderr)[-3000:]


def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_1804_07135_amd", "csrc")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc]
    srcs = [os.path.join(ROOT, "tests", "host", "plan_sanitize.cpp"), os.path.join(csrc, "ssm_api.hip"),
            os.path.join(csrc, "ssm_kernels.hip")]
    objs, procs = [], []
    for i, src in enumerate(srcs):
        obj = str(tmp_path / f"o{i}.o")
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc] + common + ["-c", src, "-o", obj],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-3000:]
    exe = str(tmp_path / "plan_sanitize")
    subprocess.check_call([hipcc] + common + objs + ["-o", exe], stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), (r.stdout + r.stderr)[-3000:]
