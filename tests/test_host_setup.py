"""The host-side set-up code (paper_2508_04484_amd/csrc/setup.cpp: P_N algebra,
eigen-split, DG energy operator and its integrals) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer, and run against closed forms
(tests/host/setup_check.cpp).  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_04484_amd", "csrc")


def test_setup_routines_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "setup_check")
    build = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-static-libasan", "-I", CSRC,
             os.path.join(ROOT, "tests", "host", "setup_check.cpp"),
             os.path.join(CSRC, "setup.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "0 failures" in r.stdout
