"""The host plan builder (decomp.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: a g++ build of it with a driver that plans cube
meshes (Q1 and Q2 elements, both variants, all preconditioners, uneven and
partially constrained subdomains, pressure faces) and malformed meshes.  Host code only; no GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_builder_under_asan_ubsan(tmp_path):
    exe = tmp_path / "plan_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1508_02599_amd", "csrc"),
           os.path.join(ROOT, "tests", "host_asan", "plan_driver.cpp"),
           os.path.join(ROOT, "paper_1508_02599_amd", "csrc", "decomp.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "OK (0 failures)" in r.stdout
