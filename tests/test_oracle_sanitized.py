"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, g++) and run through every entry point on small 2D and 3D grids
(oracle/sanitize_check.cpp): no memory error, no undefined behaviour, finite
results."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-o", exe,
           os.path.join(ORACLE, "sanitize_check.cpp"), os.path.join(ORACLE, "sgp_oracle.cpp")]
    subprocess.run(cmd, check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
