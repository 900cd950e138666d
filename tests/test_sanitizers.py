"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU code (no GPU): the oracle,
driven through every entry point by tests/oracle_sanitize_driver.c, and the library's host
grid logic (ljmd_host.hip, host code only) under the brick checker. Any invalid memory
access or undefined operation aborts the run."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    exe = tmp_path / "oracle_sanitize"
    subprocess.run([gcc, "-std=c99", "-O1", "-g", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
                    os.path.join(ROOT, "oracle", "oracle_md.c"), "-lm", "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip() == "ok" and "runtime error" not in r.stderr


def test_host_grid_under_sanitizers(tmp_path):
    hipcc = next((c for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc"))
                  if c and os.path.exists(c)), None)
    if hipcc is None:
        pytest.skip("hipcc is not available")
    exe = tmp_path / "host_grid_check_san"
    # sanitizers for the host code only
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *san,
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host_grid_check.cpp"),
                    os.path.join(ROOT, "paper_1308_5587_amd", "csrc", "ljmd_host.hip"),
                    "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.split()[0] == "ok" and "runtime error" not in r.stderr
