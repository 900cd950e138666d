"""Pins of the oracle's NVT integrator (Nose-Hoover thermostat in the symmetric
time-reversible splitting, the Martyna-Tobias-Klein family of the paper's MD listing,
Section "Capabilities"), against facts that hold independently of the code:

* zero coupling (tau = infinity) is the NVE step, bit for bit;
* the extended energy K + U + Q xi^2 / 2 + N_f kT eta is conserved, with an error that
  falls as dt^2 (a second-order splitting);
* the splitting is time reversible: stepping forward, negating v and xi, and stepping the
  same count returns to the start;
* free particles are all scaled by the same factor (the thermostat acts on the total
  kinetic energy only);
* the thermostat drives the time average of 2K to N_f kT with N_f = 3N - 3, and relaxes a
  hot start to the target temperature.
"""

import math

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen


def _fluid(oracle_mod, n=500, T=2.0, seed=3, dt=0.005):
    s = gen.make_lj_fluid(n, rho=0.8442, T=T, seed=seed)
    return s, oracle_mod.OracleSystem.from_spec(s, dt=dt)


def _ext_energy(o):
    U, K = o.energy()
    return U + K + o.thermostat()[2]


def test_zero_coupling_is_nve_bitwise(oracle_mod):
    s, a = _fluid(oracle_mod, n=400, T=1.2)
    b = oracle_mod.OracleSystem.from_spec(s)
    a.set_nvt(1.2, float("inf"))
    a.step(60)
    b.step(60)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.thermostat() == (0.0, 0.0, 0.0)


def test_extended_energy_conserved_second_order(oracle_mod):
    # a hot start thermostatted to kT = 1.2: K + U changes by hundreds of energy units while
    # the extended energy stays put, and its error falls as dt^2
    errs = []
    for dt in (0.004, 0.002):
        s, o = _fluid(oracle_mod, n=256, T=2.0, dt=dt)
        o.set_nvt(1.2, 0.5)
        h0 = _ext_energy(o)
        e0 = sum(o.energy())
        m = int(round(0.004 / dt))
        worst = 0.0
        for _ in range(16):
            o.step(25 * m)
            worst = max(worst, abs(_ext_energy(o) - h0))
        moved = abs(sum(o.energy()) - e0)
        assert moved > 50.0 * worst  # the thermostat did exchange energy
        errs.append(worst)
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.0, errs


def test_time_reversible(oracle_mod):
    s, o = _fluid(oracle_mod, n=300, T=1.6, seed=5)
    o.set_nvt(1.2, 0.3)
    x0, v0, i0, _ = o.state()
    o.step(40)
    xi, eta, _ = o.thermostat()
    assert abs(xi) > 1e-3
    o.negate_velocities()
    o.set_thermostat(-xi, eta)
    o.step(40)
    x1, v1, i1, _ = o.state()
    d = (x1 + i1 * s.box) - (x0 + i0 * s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v1 + v0).max() < 1e-9
    xi1, eta1, _ = o.thermostat()
    assert abs(xi1) < 1e-10 and abs(eta1) < 1e-10


def test_free_particles_scaled_together(oracle_mod):
    rng = np.random.default_rng(7)
    n = 64
    box = np.array([12.0, 12.0, 12.0])
    pos = rng.uniform(0, 12.0, (n, 3))
    vel = rng.normal(0, 1.5, (n, 3))
    o = oracle_mod.OracleSystem(box, pos, vel, np.zeros(n, np.int32), 1, [(0, 0, 0.0, 1.0, 2.5)])
    o.set_nvt(1.0, 0.2)
    K0 = 0.5 * (vel ** 2).sum()
    h0 = K0
    for _ in range(5):
        o.step(37)
        _, v, _, _ = o.state()
        c = v / vel
        assert np.abs(c - c[0, 0]).max() < 1e-13 * abs(c[0, 0])
        _, K = o.energy()
        # no potential: K + Q xi^2 / 2 + N_f kT eta is conserved to the splitting error
        assert abs(K + o.thermostat()[2] - h0) < 2e-3 * h0
    assert abs(o.thermostat()[0]) > 1e-3


def test_mean_kinetic_energy_small_system(oracle_mod):
    # eight particles in a dilute box: N_f = 21, not 24; the thermostat drives the time
    # average of 2K to N_f kT whatever the dynamics (the time average of dxi/dt vanishes)
    rng = np.random.default_rng(11)
    n = 8
    box = np.array([7.0, 7.0, 7.0])
    side = np.arange(2) * 3.5 + 1.75
    pos = np.stack(np.meshgrid(side, side, side, indexing="ij"), -1).reshape(-1, 3)
    vel = rng.normal(0, 1.0, (n, 3))
    vel -= vel.mean(0)
    o = oracle_mod.OracleSystem(box, pos, vel, np.zeros(n, np.int32), 1, [(0, 0, 1.0, 1.0, 2.5)])
    kT = 1.5
    o.set_nvt(kT, 0.2)
    samples = []
    for _ in range(3000):
        o.step(2)
        samples.append(2.0 * o.energy()[1])
    mean2k = np.mean(samples[500:])
    assert abs(mean2k / ((3 * n - 3) * kT) - 1.0) < 0.04, mean2k / ((3 * n - 3) * kT)


def test_hot_start_relaxes_to_target(oracle_mod):
    s, o = _fluid(oracle_mod, n=256, T=2.0, seed=9)
    o.set_nvt(1.2, 0.25)
    temps = []
    for _ in range(120):
        o.step(20)
        temps.append(2.0 * o.energy()[1] / (3 * 256 - 3))
    late = np.mean(temps[60:])
    assert abs(late - 1.2) < 0.05, late
    assert temps[0] > 1.4


def test_nvt_argument_errors(oracle_mod):
    s, o = _fluid(oracle_mod, n=100, T=1.2)
    for kT, tau in ((0.0, 1.0), (-1.0, 1.0), (1.2, 0.0), (1.2, -1.0), (float("nan"), 1.0)):
        with pytest.raises(oracle_mod.OracleError):
            o.set_nvt(kT, tau)
