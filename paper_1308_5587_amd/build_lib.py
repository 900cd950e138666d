"""Compile libljmd.so (HIP, gfx950) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libljmd.so")
LIB_DEBUG = os.path.join(HERE, "libljmd_debug.so")  # LJMD_DEBUG_CHECKS=1: device checks
SOURCES = ["ljmd_kernels.hip", "ljmd_force_lj.hip", "ljmd_force_mie.hip", "ljmd_force_gauss.hip",
           "ljmd_force_yukawa.hip", "ljmd_force_lj_sf.hip", "ljmd_force_mie_sf.hip",
           "ljmd_force_gauss_sf.hip", "ljmd_force_yukawa_sf.hip", "ljmd_force_glist.hip",
           "ljmd_bvh.hip", "ljmd_host.hip", "ljmd_system.hip", "ljmd_batch.hip"]

# -ffp-contract=off: the distance arithmetic must not be fused (explicit fma elsewhere).
# -packed-fp32-ops: keep the compiler from emitting packed FP32 instructions.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, debug: bool = False) -> str:
    """Compile the sources into the in-tree libljmd.so, or with debug into libljmd_debug.so,
    the same sources with the device checks of LJMD_DEBUG_CHECKS compiled in."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(HERE, "_build_debug" if debug else "_build")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    flags = HIPFLAGS + (["-DLJMD_DEBUG_CHECKS=1"] if debug else [])

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose:
            sys.stderr.write(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(compile_one, srcs))
    out = LIB_DEBUG if debug else LIB
    tmp = out + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, debug="--debug" in sys.argv[1:]))
