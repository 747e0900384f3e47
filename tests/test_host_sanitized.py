"""The library's host-only logic under AddressSanitizer and UndefinedBehaviorSanitizer:
workspace and interaction-list layouts, the server's first-fit arena and its first-come
first-served admission (paper_1109_5190_amd/csrc/bh_host.h, which holds no HIP code), driven
by a C++ program that checks their invariants against plain reference models.  Built with the
host compiler and its sanitizers; CPU only."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_logic_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "host_sanitized"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
           str(ROOT / "tests" / "host_sanitize_driver.cpp"), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "sanitizer" in res.stderr.lower():
        pytest.skip("the host compiler has no sanitizer runtime")
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "all cases ok" in run.stdout
