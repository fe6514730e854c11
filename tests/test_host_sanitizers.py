"""The plan builder's host code (plan.cpp: stencil weights, spectra, D^e tables, frame
spectra, constraint and broken-bond validation, crack -> bonds, surface factors) built for
the CPU with AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only, HIP calls
replaced by host-memory stand-ins in tests/sanitize/hip_host_stub.cpp) and driven through
the C ABI by tests/sanitize/plan_host_driver.cpp: no sanitizer report, every call as
expected."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_plan_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "plan_host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wno-unused-result", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "paper_2301_11828_amd", "csrc", "plan.cpp"),
           os.path.join(HERE, "sanitize", "hip_host_stub.cpp"),
           os.path.join(HERE, "sanitize", "plan_host_driver.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "0 failed checks" in r.stdout
