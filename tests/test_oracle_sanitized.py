"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C driver calls every
entry point on small and degenerate inputs (one to three bodies, coincident bodies,
duplicate keys at the depth limit, distant clusters; leaf sizes 1, 8 and 64; theta 0,
0.6 and huge; softened and unsoftened; every opening radius, the quadrupole and the
group walk), built with the sanitizers on the host compiler.  CPU only."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           str(ROOT / "tests" / "oracle_sanitize_driver.c"), str(ROOT / "oracle" / "bh_oracle.c"),
           "-o", str(exe), "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "sanitizer" in res.stderr.lower():
        pytest.skip("the host compiler has no sanitizer runtime")
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, OMP_NUM_THREADS="1", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "all cases ok" in run.stdout
