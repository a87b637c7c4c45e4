"""The CPU oracle under host sanitizers: oracle/arsel_oracle.c built by gcc
with AddressSanitizer and UndefinedBehaviorSanitizer (no recovery) together
with tests/sanitize/oracle_driver.c, which calls every entry point on small
inputs and their edge cases (sequential build: no OpenMP)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    sanitize = "-fsanitize=" + ",".join(("address", "undefined"))
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           sanitize, "-fno-sanitize-recover=all", "-Wall",
           os.path.join(ROOT, "oracle", "arsel_oracle.c"),
           os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "sanitized oracle run ok" in r.stdout
