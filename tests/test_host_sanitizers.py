"""The library's host-only code (momentum rules, lambda map, batched schedule,
tuning-cache file; paper_1912_03514_amd/csrc/host.cpp) built with the host
compiler under AddressSanitizer and UndefinedBehaviorSanitizer, and exercised by
tests/host_checks.cpp: random problem sets for the scheduler, a cache round
trip, malformed and randomly corrupted cache files.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = os.environ.get("CXX", "g++")


@pytest.mark.skipif(shutil.which(CXX) is None, reason="no host C++ compiler")
def test_host_code_under_sanitizers(tmp_path):
    exe = tmp_path / "host_checks"
    cmd = [CXX, "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_checks.cpp"),
           os.path.join(ROOT, "paper_1912_03514_amd", "csrc", "host.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
