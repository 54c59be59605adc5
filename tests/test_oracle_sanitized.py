"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a build of the same source with both sanitizers runs the oracle's
own test files in a child process; any out-of-bounds access, use after free
or undefined behaviour aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def test_oracle_tests_pass_under_asan_and_ubsan():
    from oracle import build as ob
    lib = ob.build(sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    env = dict(os.environ, CQ_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    files = ["tests/test_oracle_codec.py", "tests/test_oracle_sv.py", "tests/test_oracle_values.py",
             "tests/test_oracle_zero_chunks.py", "tests/test_oracle_const_chunks.py", "tests/test_fused_plan.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
                        *files], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
