"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (tests/sanitize/oracle_driver.c) calls every oracle entry point on a
small cloud; the instrumented build aborts on any out-of-bounds access,
use after free, leak or undefined operation."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-ffp-contract=off", os.path.join(ROOT, "oracle", "gmm_oracle.c"),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle driver ok" in r.stdout
