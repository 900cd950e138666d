"""NVT on the GPU (ljmd_set_nvt: Nose-Hoover thermostat in the symmetric splitting of the
paper's MD listing) through the C ABI, against the CPU FP64 oracle on identical seeded
inputs: one step within 1e-12 (state) and 1e-10 (forces), 100 steps within 1e-8, the
thermostat variables alike; zero coupling equals the NVE path bit for bit; time reversal;
checkpoint and resume; overflow recovery; the paper's benchmark liquid (N = 64,000,
density 0.382, r_cut = 3.0, kT = 1.2)."""

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen
from parity import max_norm_rel, print_case, unwrapped

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ljmd_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1308_5587_amd import ljmd

    ljmd.load()
    return ljmd


def _compare(o, g, box, tol_x, tol_f, tol_th):
    po, vo, io, so = o.state()
    pg, vg, ig, sg = g.state()
    assert so == sg
    dx = np.abs(unwrapped(pg, ig, box) - unwrapped(po, io, box)).max()
    dv = np.abs(vg - vo).max()
    assert dx < tol_x and dv < tol_x, (dx, dv)
    assert max_norm_rel(g.forces(), o.forces()) < tol_f
    xo, eo, _ = o.thermostat()
    xg, eg, _ = g.thermostat()
    assert abs(xg - xo) < tol_th and abs(eg - eo) < tol_th, (xg, xo, eg, eo)


@pytest.mark.parametrize("precision_graph", [("fp64", 64), ("fp64", -1)])
def test_nvt_one_and_hundred_steps(ljmd_mod, oracle_mod, precision_graph):
    _, graph = precision_graph
    print_case(f"nvt 1 and 100 steps n=4000 graph={graph}")
    s = gen.make_lj_fluid(4000, T=2.0, seed=1)  # hot start: the thermostat works hard
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s, graph_steps=graph)
    o.set_nvt(1.2, 0.5)
    g.set_nvt(1.2, 0.5)
    o.step(1)
    g.step(1)
    _compare(o, g, s.box, 1e-12, 1e-10, 1e-12)
    o.step(99)
    g.step(99)
    _compare(o, g, s.box, 1e-8, 1e-8, 1e-8)
    U, K = g.energy()
    Uo, Ko = o.energy()
    assert abs(K - Ko) < 1e-8 * abs(Ko) and abs(U - Uo) < 1e-8 * abs(Uo)
    assert abs(g.thermostat()[0]) > 1e-2  # the thermostat is active
    assert g.stats()["rebuilds"] >= 5


def test_nvt_mixed_tracks_oracle(ljmd_mod, oracle_mod):
    print_case("nvt mixed precision n=4000")
    s = gen.make_lj_fluid(4000, T=2.0, seed=2)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s, precision="mixed")
    o.set_nvt(1.2, 0.5)
    g.set_nvt(1.2, 0.5)
    o.step(1)
    g.step(1)
    assert max_norm_rel(g.forces(), o.forces()) < 1e-5
    o.step(99)
    g.step(99)
    po, _, io, _ = o.state()
    pg, _, ig, _ = g.state()
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < 1e-3
    assert abs(g.thermostat()[0] - o.thermostat()[0]) < 1e-3


def test_zero_coupling_equals_nve_bitwise(ljmd_mod):
    print_case("nvt with tau = inf equals the NVE path")
    s = gen.make_lj_fluid(3000, T=1.2, seed=4)
    a = ljmd_mod.System.from_spec(s, threads_per_particle=2, block_size=256)
    b = ljmd_mod.System.from_spec(s, threads_per_particle=2, block_size=256)
    a.set_nvt(1.2, float("inf"))
    for k in (1, 70, 3):
        a.step(k)
        b.step(k)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.forces(), b.forces())
    assert a.thermostat() == (0.0, 0.0, 0.0)


def test_nvt_time_reversal(ljmd_mod):
    print_case("nvt time reversal")
    s = gen.make_lj_fluid(2000, T=1.6, seed=5)
    g = ljmd_mod.System.from_spec(s)
    g.set_nvt(1.2, 0.3)
    x0, v0, i0, _ = g.state()
    g.step(40)
    xi, eta, _ = g.thermostat()
    g.negate_velocities()
    g.set_thermostat(-xi, eta)
    g.step(40)
    x1, v1, i1, _ = g.state()
    assert np.abs(unwrapped(x1, i1, s.box) - unwrapped(x0, i0, s.box)).max() < 1e-9
    assert np.abs(v1 + v0).max() < 1e-9
    xi1, eta1, _ = g.thermostat()
    assert abs(xi1) < 1e-10 and abs(eta1) < 1e-10


def test_nvt_checkpoint_resume_and_overflow(ljmd_mod, oracle_mod):
    print_case("nvt checkpoint/resume and list overflow")
    s = gen.make_lj_fluid(3000, T=1.8, seed=6)
    a = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128)
    a.set_nvt(1.2, 0.5)
    a.step(30)
    pos, vel, img, st = a.state()
    xi, eta, _ = a.thermostat()
    b = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128)
    b.set_nvt(1.2, 0.5)
    b.set_state(pos, vel, img, st)
    b.set_thermostat(xi, eta)
    a.set_state(pos, vel, img, st)  # the same forced rebuild on both
    a.set_thermostat(xi, eta)
    a.step(20)
    b.step(20)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.thermostat() == b.thermostat()
    # a list capacity far too small: the step is re-run after growth, thermostat included
    c = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128, nlist_capacity=16)
    d = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128)
    c.set_nvt(1.2, 0.5)
    d.set_nvt(1.2, 0.5)
    c.step(50)
    d.step(50)
    assert c.stats()["overflow_retries"] >= 1
    pc, vc, ic, _ = c.state()
    pd, vd, id_, _ = d.state()
    assert np.abs(unwrapped(pc, ic, s.box) - unwrapped(pd, id_, s.box)).max() < 1e-10
    assert np.abs(vc - vd).max() < 1e-10
    assert abs(c.thermostat()[0] - d.thermostat()[0]) < 1e-10


def test_paper_benchmark_liquid(ljmd_mod, oracle_mod):
    """The paper's LJ liquid benchmark: N = 64,000 on a 40^3 simple-cubic lattice, density
    0.382, r_cut = 3.0, NVT at kT = 1.2 (tau = 1.0 as in its MD listing), dt = 0.005."""
    print_case("paper benchmark liquid N=64000 NVT")
    s = gen.make_lj_fluid(64000, rho=0.382, T=1.2, seed=1, r_cut=3.0)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    o.set_nvt(1.2, 1.0)
    g.set_nvt(1.2, 1.0)
    assert max_norm_rel(g.forces(), o.forces()) < 1e-10
    o.step(1)
    g.step(1)
    _compare(o, g, s.box, 1e-12, 1e-10, 1e-12)
    o.step(29)
    g.step(29)
    _compare(o, g, s.box, 1e-9, 1e-9, 1e-9)
