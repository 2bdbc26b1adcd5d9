"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

tests/oracle_sanitize.c calls every oracle entry point on small inputs:
single cells of D1Q3, D2Q9 and D3Q27 in every path-length mode, and whole
lattices with extents of 1, 2 and ragged sizes in every step mode, forced,
walled and ES-BGK.  It is built with gcc together with the oracle's source,
both instrumented, and any out-of-bounds access, use after free, leak or
undefined operation ends the run with an error.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_sanitize"
    cmd = [gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", str(exe), os.path.join(ROOT, "tests", "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "eselbm_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ran clean" in res.stdout
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr
