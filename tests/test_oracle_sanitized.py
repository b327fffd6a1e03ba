"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(every check fatal), driven through every equation family, limiter mode,
degree parity and boundary kind on small meshes with every trace array
requested (tests/sanitized/oracle_driver.c).  A memory error, an undefined
operation or an error return of the oracle fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "tests", "sanitized", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "idp_ref.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-4000:])
    assert "FAIL" not in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
