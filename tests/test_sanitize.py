"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only), driven through every entry point on small random
inputs by tests/sanitize/oracle_driver.cpp."""
import os
import shutil
import subprocess
import tempfile

import pytest

from conftest import ROOT


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitized")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
               os.path.join(ROOT, "oracle", "oracle.cpp"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp"),
               "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
        res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-3000:]
        assert "ok" in res.stdout
