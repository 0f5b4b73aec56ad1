"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU:
tests/native/host_checks.cpp links every translation unit of libhipsso (host code sanitized;
the device code is built but never launched) and runs the C ABI's argument-error paths, the host-only entry points and the
debug-mode pattern checker on correct and on corrupted patterns."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_20026_amd", "csrc")
OUT = os.path.join(ROOT, "paper_2407_20026_amd", "_build", "host_checks")


def _sources():
    from paper_2407_20026_amd import build
    return [os.path.join(CSRC, s) for s in build.SOURCES]


def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    from paper_2407_20026_amd import build
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = [build.hipcc(), "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
           f"--offload-arch={build.ARCH}", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *_sources(), os.path.join(ROOT, "tests", "native", "host_checks.cpp"), "-o", OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(f"build failed:\n{r.stderr[-4000:]}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([OUT], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("ok (0 failures)")
