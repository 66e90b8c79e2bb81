"""The C ABI's host code (argument checks, status codes, workspace and
stack layout of api.cpp) built for the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer and driven through every entry point with valid
and invalid arguments (tests/asan/abi_driver.cpp). The kernel launchers are
replaced by host stand-ins (tests/asan/stub_launchers.cpp) that check every
plane a kernel would read or write against the caller's buffers, so an
overrun in the layout arithmetic fails the run. No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "abi_driver")
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                 "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", flag]
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", *san,
           "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "paper_1811_02308_amd", "csrc", "api.cpp"),
           os.path.join(ROOT, "tests", "asan", "stub_launchers.cpp"),
           os.path.join(ROOT, "tests", "asan", "abi_driver.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failed checks, 0 out-of-buffer planes" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
