"""The oracle built with the address and undefined-behaviour sanitizers
(gcc), driven through every boundary kind and entry point by
tests/oracle_sanitized_driver.c: no sanitizer report, every lattice
finite.  Host code only; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    subprocess.check_call(
        ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall",
         "-o", exe, os.path.join(HERE, "oracle_sanitized_driver.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout
