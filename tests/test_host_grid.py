"""Host logic of the brick tables (no GPU): the library's own make_grid, compiled with the
checker tests/host_grid_check.cpp, over random box shapes, densities, cutoffs and skins.

The checker verifies that each brick is a block of cells, that an axis is marked for centring
exactly when it holds at least (brick cells + 2) cells, that the stored centre is the middle
of the brick, and, by sampling particles of the brick (moved by less than skin/2 since the
build) with partners closer than r_cut, that centring both on the brick reproduces the
minimum-image difference on every centred axis and the plain difference on every wrap-free
axis. These are the facts the force kernel's plain differences rest on."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_brick_centring_and_wrap_free_axes(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc is not available")
    exe = tmp_path / "host_grid_check"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host_grid_check.cpp"),
                    os.path.join(ROOT, "paper_1308_5587_amd", "csrc", "ljmd_host.hip"),
                    "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:]
    ok, bricks, pairs = r.stdout.split()[:3]
    assert ok == "ok" and int(bricks) > 10000 and int(pairs) > 200000
