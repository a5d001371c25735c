"""The library's host-side CSR checks (the validation behind
ef_validate_csr and the bounds check every load runs) under AddressSanitizer
and UndefinedBehaviorSanitizer (no GPU needed).

``csrc/csr_check.cpp`` is built from source together with a test driver
(``tests/native/csr_check_driver.cpp``) that hands it exact-size heap arrays:
malformed CSRs with known statuses, and 20000 random garbage CSRs. A read
outside any array, signed overflow or other undefined behaviour aborts the
run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_00606_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_csr_checks_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "csr_check_asan")
        r = subprocess.run(
            ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             os.path.join(ROOT, "tests", "native", "csr_check_driver.cpp"),
             os.path.join(CSRC, "csr_check.cpp"), "-o", exe],
            capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.startswith("ok"), r.stdout
