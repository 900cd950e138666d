"""The debug build (LJMD_DEBUG_CHECKS=1: device checks of cell, slot, tile and list indices
and of dangerous builds) through the C ABI: on every path (cell and tree lists, both
precisions, small boxes with the branch-form minimum image, NVT with thermo samples, a
batch) no check fails, and the results are bit for bit those of the release build. The
debug build runs in a child process, since a process loads one library."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from parity import print_case

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import json, sys, hashlib
sys.path.insert(0, ROOT)
import numpy as np
import torch
from paper_1308_5587_amd import ljmd, inputs as gen
ljmd.load()
out = {"version": ljmd.version()}

def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()

def run(name, spec, steps, **kw):
    nlist = kw.pop("nlist", None)
    nvt = kw.pop("nvt", None)
    thermo = kw.pop("thermo", None)
    g = ljmd.System.from_spec(spec, **kw)
    if nlist:
        g.set_nlist(nlist)
    if nvt:
        g.set_nvt(*nvt)
    if thermo:
        g.set_thermo(*thermo)
    g.step(steps)
    pos, vel, img, st = g.state()
    U, K = g.energy()
    out[name] = digest(pos, vel, img, g.forces(), np.array([U, K]), g.thermo() if thermo else np.zeros(0))
    g.close()

run("fluid_fp64", gen.make_lj_fluid(4000, T=1.2, seed=11), 200)
run("fluid_mixed", gen.make_lj_fluid(4000, T=1.2, seed=12), 60, precision="mixed")
run("ka_mixed", gen.make_ka_mixture(4000, seed=13), 60, precision="mixed")
run("small_box", gen.make_lj_fluid(216, T=1.2, seed=14), 60)
run("nvt_thermo", gen.make_lj_fluid(4000, T=2.0, seed=15), 40, nvt=(1.2, 0.5), thermo=(10, 8))
run("tree", gen.make_colloid_mixture(n_large_side=4, sigma_l=3.0), 30, nlist="tree")

specs = [gen.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)
         for p in gen.make_replica_specs(count=8, seed=16, n_lo=256, n_hi=2048)]
b = ljmd.Batch(256 << 20, 8, precision="mixed", block_steps=50, threads_per_particle=2,
               block_size=256)
slots = [b.admit(s, 100) for s in specs]
pending = set(slots)
while pending:
    b.run_block()
    pending -= set(b.poll())
out["batch"] = digest(*[np.concatenate([np.ravel(b.read(s)[k]) for k in ("pos", "vel", "forces", "virial")])
                         for s in slots])
b.close()
print(json.dumps(out))
'''


def _run(debug):
    env = dict(os.environ)
    env.pop("LJMD_DEBUG_CHECKS", None)
    if debug:
        env["LJMD_DEBUG_CHECKS"] = "1"
    r = subprocess.run([sys.executable, "-c", SCRIPT.replace("ROOT", repr(ROOT))], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_debug_build_checks_pass_and_change_nothing():
    print_case("debug build: fluid, mixed, KA, small box, NVT + thermo, tree, batch")
    if not os.path.exists(os.path.join(ROOT, "paper_1308_5587_amd", "libljmd_debug.so")):
        pytest.fail("libljmd_debug.so is missing: build it with build_lib.build(debug=True)")
    dbg = _run(True)
    rel = _run(False)
    assert "debug checks" in dbg["version"] and "debug" not in rel["version"]
    for k in rel:
        if k != "version":
            assert dbg[k] == rel[k], k
