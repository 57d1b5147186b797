"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
every entry point on small grids, all 25 side pairings, Poisson and
Helmholtz, with exactly sized arrays (tests/oracle_sanitize_driver.c).  Any
out-of-bounds access, use of freed memory, signed overflow or other undefined
behaviour stops the run with a report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE,
           os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ORACLE, "mg_oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "failures: 0" in r.stdout
    assert r.stdout.count(" ok") >= 300
