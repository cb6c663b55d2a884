"""The oracle under AddressSanitizer (with leak detection) and
UndefinedBehaviorSanitizer on the CPU: tests/csrc/oracle_sanitize_driver.c
runs the sweeps in every mode and order, the per-link pass, replica
exchange, the reconstruction and the network on small lattices; any
out-of-bounds access, use after free, leak or undefined operation aborts
the run."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "or_san")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "llr_oracle.c"), os.path.join(HERE, "csrc", "oracle_sanitize_driver.c"),
           "-o", exe, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "sanitize" in b.stderr:
        pytest.skip("gcc without sanitizer runtimes: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "oracle sanitizer run" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
