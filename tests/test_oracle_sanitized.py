"""The serial oracle and the multi-threaded CPU baseline built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only, g++) and
run on seeded random meshes by tests/sanitize_driver.cpp: any out-of-bounds
access, use after free, leak or undefined operation in either file fails
the test, as does a disagreement between the two or a broken re-index
identity."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.slow
def test_oracle_and_parallel_baseline_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(
        ["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         os.path.join(HERE, "sanitize_driver.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp"),
         os.path.join(ROOT, "oracle", "parallel_cpu.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "300"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "300 cases, 0 failures" in r.stdout
