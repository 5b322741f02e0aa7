"""libpf's host setup and C ABI built with AddressSanitizer and UBSan
(g++, host code only, a stub device layer) and driven through valid,
batched, multi-grid and malformed networks.  CPU only."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_11880_amd", "csrc")
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "host_sanitize")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "pf_host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "pf_setup.cpp"), os.path.join(CSRC, "pf_api.cpp"),
           os.path.join(HERE, "stub_device.cpp"), os.path.join(HERE, "sanitize_main.cpp"),
           "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
