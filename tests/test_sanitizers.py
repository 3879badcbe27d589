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


def test_host_api_under_asan_and_ubsan(tmp_path):
    """fdtd_api.hip with AddressSanitizer and UBSan on its host code, linked
    with the library's kernel objects: the validation of every descriptor
    field, workspace sizing with and without conducting cells, create's
    argument checks and the checkpoint planner run clean (no GPU needed)."""
    root = os.path.dirname(HERE)
    build = os.path.join(root, "paper_2412_12360_amd", "_build")
    hipcc = "/opt/rocm/bin/hipcc"
    kern = [os.path.join(build, f + ".hip.o") for f in ("kern_aux", "kern_naive", "kern_tb", "kern_tb_rev")]
    if not os.path.exists(hipcc) or not all(os.path.exists(k) for k in kern):
        pytest.skip("needs hipcc and the built kernel objects")
    inc = os.path.join(root, "include")
    api = tmp_path / "api.o"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", inc,
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-c", os.path.join(root, "paper_2412_12360_amd", "csrc", "fdtd_api.hip"), "-o", str(api)],
                          stderr=subprocess.DEVNULL)
    drv = tmp_path / "drv.o"
    subprocess.check_call(["/opt/rocm/bin/amdclang++", "-O1", "-g", "-std=c++17", "-I", inc, "-D__HIP_PLATFORM_AMD__",
                           "-fsanitize=address,undefined", "-c", os.path.join(HERE, "sanitize", "api_driver.cpp"),
                           "-o", str(drv)])
    exe = tmp_path / "api_asan"
    subprocess.check_call([hipcc, "-fsanitize=address,undefined", "-fno-gpu-sanitize", str(drv), str(api), *kern,
                           "-o", str(exe)], stderr=subprocess.DEVNULL)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count("case ") == 12 and "lossy 0" in r.stdout
