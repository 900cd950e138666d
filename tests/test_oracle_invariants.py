"""Pin the CPU oracle to closed forms and conservation laws that do not depend on it:

* the LJ pair function: minimum at 2^(1/6) sigma with U = -eps and F = 0, the values at
  r = sigma and r = r_cut, and F = -du/dr by central difference;
* perfect simple-cubic lattices: zero force by symmetry, and energy, virial and list
  neighbour counts from lattice sums over integer shells;
* Newton's third law (net force ~ 0), the virial as the strain derivative of the energy;
* the integrator: free flight with wraps and image counters, time reversibility, momentum
  conservation, energy fluctuation scaling as dt^2, bounded NVE drift;
* error paths: box too small, incomplete pair table, overlapping particles.
"""

import itertools
import math

import numpy as np
import pytest

from brute import lj_pair
from paper_1308_5587_amd import inputs as gen


def _two(oracle_mod, r, eps=1.0, sig=1.0, rc=2.5, L=10.0, axis=0):
    box = np.array([L, L, L])
    pos = np.full((2, 3), 1.0)
    pos[1, axis] += r
    vel = np.zeros((2, 3))
    o = oracle_mod.OracleSystem(box, pos, vel, np.zeros(2, np.int32), 1,
                                [(0, 0, eps, sig, rc)])
    return o


def test_lj_minimum(oracle_mod):
    rmin = 2.0 ** (1.0 / 6.0)
    o = _two(oracle_mod, rmin, rc=1e3 / 1e3 * 2.5)
    F = o.forces()
    U, _ = o.energy()
    shift = 4.0 * ((1 / 2.5) ** 12 - (1 / 2.5) ** 6)
    assert abs(U - (-1.0 - shift)) < 1e-14
    assert np.abs(F).max() < 1e-12
    assert abs(-0.983683108864 - U) < 1e-11  # shifted value at the minimum


@pytest.mark.parametrize("r,u_ref,f_ref", [
    (1.0, 0.016316891136, 24.0),                 # u(sigma) = -U_LJ(r_cut); |F| = 24 eps/sigma
    (2.0, -0.045206546364, -0.181640625),        # 4(2^-12 - 2^-6) - shift; 24(2^-11 - 2^-6)/2
])
def test_pair_values(oracle_mod, r, u_ref, f_ref):
    o = _two(oracle_mod, r)
    F = o.forces()
    U, _ = o.energy()
    assert abs(U - u_ref) < 1e-11
    # force on particle 0 from particle 1 placed at +r along x: -f_ref along x
    assert abs(F[0, 0] + f_ref) < 1e-12 and abs(F[1, 0] - f_ref) < 1e-12
    W = o.virial()
    assert abs(W[0] - r * f_ref) < 1e-12 and np.abs(W[1:]).max() < 1e-14


def test_cutoff_is_strict_and_force_unshifted(oracle_mod):
    o = _two(oracle_mod, 2.5)
    assert np.abs(o.forces()).max() == 0.0 and o.energy()[0] == 0.0
    o = _two(oracle_mod, 2.5 - 1e-9)
    f = o.forces()[1, 0]
    assert abs(f - (-0.038999477453)) < 1e-9  # force just inside r_cut is not shifted to 0
    assert abs(o.energy()[0]) < 1e-9


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_force_is_minus_energy_gradient(oracle_mod, axis):
    for r in [0.95, 1.1, 1.5, 2.2]:
        h = 1e-6
        up = _two(oracle_mod, r + h, axis=axis).energy()[0]
        dn = _two(oracle_mod, r - h, axis=axis).energy()[0]
        f = _two(oracle_mod, r, axis=axis).forces()[1, axis]
        assert abs(f - (-(up - dn) / (2 * h))) < 1e-6 * max(1.0, abs(f))
        assert abs(f - lj_pair(r)[1]) < 1e-12 * max(1.0, abs(f))


def test_pair_across_periodic_boundary(oracle_mod):
    box = np.array([8.0, 9.0, 10.0])
    pos = np.array([[0.2, 4.0, 5.0], [7.3, 4.0, 5.0]])  # separated by 0.9 through x = 0
    o = oracle_mod.OracleSystem(box, pos, np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                                [(0, 0, 1.0, 1.0, 2.5)])
    F = o.forces()
    _, f = lj_pair(0.9)
    # particle 0 is pushed towards +x (away from its image neighbour on the -x side)
    assert abs(F[0, 0] - f) < 1e-9 and abs(F[1, 0] + f) < 1e-9


def _shells(a, r_max):
    """Lattice sum helper: {|n|^2: count} over integer vectors with 0 < |n| a < r_max."""
    k = int(math.ceil(r_max / a)) + 1
    cnt = {}
    for n in itertools.product(range(-k, k + 1), repeat=3):
        s = n[0] ** 2 + n[1] ** 2 + n[2] ** 2
        if s > 0 and math.sqrt(s) * a < r_max:
            cnt[s] = cnt.get(s, 0) + 1
    return cnt


@pytest.mark.parametrize("side,a", [(10, 2.0), (16, (1.0 / 0.8442) ** (1.0 / 3.0))])
def test_perfect_sc_lattice(oracle_mod, side, a):
    n = side ** 3
    L = side * a
    idx = np.array(list(itertools.product(range(side), repeat=3)), dtype=np.float64)
    pos = (idx + 0.5) * a
    o = oracle_mod.OracleSystem(np.array([L, L, L]), pos, np.zeros((n, 3)),
                                np.zeros(n, np.int32), 1, [(0, 0, 1.0, 1.0, 2.5)])
    F = o.forces()
    assert np.abs(F).max() < 1e-10
    pe = 0.0
    wtr = 0.0
    for s2, z in _shells(a, 2.5).items():
        r = math.sqrt(s2) * a
        u, f = lj_pair(r)
        pe += 0.5 * z * u
        wtr += 0.5 * z * r * f
    U, _ = o.energy()
    W = o.virial()
    assert abs(U / n - pe) < 1e-11
    assert abs((W[0] + W[3] + W[5]) / n - wtr) < 1e-11
    assert np.abs(W[[1, 2, 4]]).max() < 1e-9 * n
    zl = sum(_shells(a, 2.9).values())
    p, _ = o.pairs()
    assert len(p) * 2 == n * zl
    if side == 10:   # the paper's example system: SC a = 2.0, n = 10
        assert abs(U / n - (-0.135619639092)) < 1e-11 and zl == 18
    else:
        assert abs(U / n - (-4.763345567633)) < 1e-9 and zl == 80


def test_newton_third_law(oracle_mod):
    s = gen.make_lj_fluid(4000, seed=1)
    o = oracle_mod.OracleSystem.from_spec(s)
    o.step(20)
    F = o.forces()
    frms = math.sqrt(np.mean(np.sum(F * F, axis=1)))
    assert np.linalg.norm(F.sum(axis=0)) <= 1e-12 * math.sqrt(s.n) * frms


@pytest.mark.parametrize("comp,axis", [(0, 0), (3, 1), (5, 2)])
def test_virial_is_strain_derivative(oracle_mod, comp, axis):
    s = gen.make_lj_fluid(400, rho=0.8442, seed=9)
    o0 = oracle_mod.OracleSystem.from_spec(s)
    o0.step(30)  # leave the lattice so that no pair sits on a symmetric shell
    pos, vel, _, _ = o0.state()
    W = o0.virial()

    def energy(lam):
        sc = np.ones(3)
        sc[axis] += lam
        o = oracle_mod.OracleSystem(s.box * sc, pos * sc, vel, s.type, 1, s.pairs)
        return o.energy()[0]

    h = 1e-7
    dU = (energy(h) - energy(-h)) / (2 * h)
    assert abs(W[comp] + dU) < 1e-5 * max(1.0, abs(W[comp]))


def test_free_flight_wraps_and_images(oracle_mod):
    rng = np.random.default_rng(4)
    n = 50
    box = np.array([7.0, 8.0, 9.0])
    pos = rng.uniform(0, 1, (n, 3)) * box
    vel = rng.normal(0, 30.0, (n, 3))
    o = oracle_mod.OracleSystem(box, pos, vel, np.zeros(n, np.int32), 1, [(0, 0, 0.0, 1.0, 2.5)])
    steps = 200
    o.step(steps)
    x, v, img, st = o.state()
    assert st == steps
    assert np.array_equal(v, vel)
    assert np.all(x >= 0) and np.all(x < box)
    unwrapped = x + img * box
    expect = pos + steps * 0.005 * vel
    assert np.abs(unwrapped - expect).max() < 1e-9
    assert np.abs(img).max() >= 1


def test_time_reversibility(oracle_mod):
    s = gen.make_lj_fluid(500, seed=3)
    o = oracle_mod.OracleSystem.from_spec(s)
    o.step(50)
    x, v, img, _ = o.state()
    o2 = oracle_mod.OracleSystem(s.box, x + img * s.box, -v, s.type, 1, s.pairs)
    o2.step(50)
    x2, v2, img2, _ = o2.state()
    back = x2 + img2 * s.box
    assert np.abs(back - s.pos).max() < 1e-9
    assert np.abs(-v2 - s.vel).max() < 1e-9


def test_momentum_conserved(oracle_mod):
    s = gen.make_lj_fluid(1000, seed=2)
    o = oracle_mod.OracleSystem.from_spec(s)
    o.step(100)
    _, v, _, _ = o.state()
    assert np.abs(v.sum(axis=0)).max() < 1e-10


def _energy_series(oracle_mod, s, dt, nsteps, every):
    o = oracle_mod.OracleSystem.from_spec(s, dt=dt)
    out = []
    for _ in range(nsteps // every):
        o.step(every)
        u, k = o.energy()
        out.append(u + k)
    return np.array(out)


def test_energy_fluctuation_scales_as_dt_squared(oracle_mod):
    s = gen.make_lj_fluid(256, rho=0.7, T=1.0, seed=12)
    o = oracle_mod.OracleSystem.from_spec(s)
    o.step(400)  # melt the lattice first
    x, v, img, _ = o.state()
    eq = gen.LJSystemSpec(s.box, x, v, s.type, 1, s.pairs)
    e1 = _energy_series(oracle_mod, eq, 0.004, 500, 5)
    e2 = _energy_series(oracle_mod, eq, 0.002, 1000, 10)
    ratio = np.std(e1) / np.std(e2)
    assert 3.0 < ratio < 5.0


def test_nve_drift_small(oracle_mod):
    s = gen.make_lj_fluid(500, seed=6)
    o = oracle_mod.OracleSystem.from_spec(s)
    u0, k0 = o.energy()
    o.step(1000)
    u1, k1 = o.energy()
    # |dE| per atom per tau over 5 tau stays small for dt = 0.005
    assert abs((u1 + k1) - (u0 + k0)) / s.n / 5.0 < 1e-3


def test_error_paths(oracle_mod):
    o_err = oracle_mod.OracleError
    # box too small for r_cut + skin
    with pytest.raises(o_err):
        o = oracle_mod.OracleSystem(np.array([5.0, 5.0, 5.0]), np.ones((2, 3)),
                                    np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                                    [(0, 0, 1.0, 1.0, 2.5)])
        o.compute()
    # incomplete pair table
    o = oracle_mod.OracleSystem(np.array([9.0] * 3), np.ones((2, 3)), np.zeros((2, 3)),
                                np.array([0, 1], np.int32), 2, [(0, 0, 1.0, 1.0, 2.5)])
    with pytest.raises(o_err):
        o.compute()
    # exact overlap gives a non-finite force
    o = oracle_mod.OracleSystem(np.array([9.0] * 3), np.ones((2, 3)), np.zeros((2, 3)),
                                np.zeros(2, np.int32), 1, [(0, 0, 1.0, 1.0, 2.5)])
    with pytest.raises(o_err):
        o.compute()
    # type index out of range
    with pytest.raises(o_err):
        oracle_mod.OracleSystem(np.array([9.0] * 3), np.ones((2, 3)), np.zeros((2, 3)),
                                np.array([0, 3], np.int32), 2, [])


def test_positions_outside_box_are_wrapped(oracle_mod):
    box = np.array([9.0, 9.0, 9.0])
    pos = np.array([[-0.5, 10.0, 20.5], [1.0, 1.0, 1.0]])
    o = oracle_mod.OracleSystem(box, pos, np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                                [(0, 0, 1.0, 1.0, 2.5)])
    x, _, img, _ = o.state()
    assert np.allclose(x[0], [8.5, 1.0, 2.5]) and np.array_equal(img[0], [-1, 1, 2])
