"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle is compiled with -fsanitize=address,undefined together with a
small driver (tests/sanitize/oracle_driver.c) that calls every entry point on
tiny problems with a CPML, point and plane sources on E and H, plain,
interpolated and energy detectors and a lossy box; any invalid access or
undefined operation aborts the run with a report.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_asan"
    src = os.path.join(HERE, "sanitize", "oracle_driver.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-ffp-contract=off", "-o", str(exe), src, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count("recon=") == 4
