"""Pins of the oracle's shifted-force option (the force less its value at r_cut, the energy
less the matching linear term, for every pair form; the survey's suggested variant for
tighter energy conservation): both vanish at r_cut, F = -du/dr by central difference, the
LJ values at r = 2 against the closed forms, and an independent numpy brute force."""

import numpy as np
import pytest

from brute import brute_fuw_style
from parity import max_norm_rel

FORMS = [("lj", (1.0, 1.0, 0.0, 0.0), 2.5), ("mie", (1.3, 1.1, 14.0, 7.0), 2.8),
         ("gauss", (2.0, 0.9, 0.0, 0.0), 2.7), ("yukawa", (1.5, 0.8, 0.0, 0.0), 2.6)]


def _two(oracle_mod, r, style, params, rc, mode="force", L=10.0):
    box = np.array([L, L, L])
    pos = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
    o = oracle_mod.OracleSystem(box, pos, np.zeros((2, 3)), np.zeros(2, np.int32), 1, [])
    o.set_pair_style(0, 0, style, params, rc)
    o.set_shift_mode(mode)
    return o


@pytest.mark.parametrize("style,params,rc", FORMS)
def test_force_and_energy_vanish_at_cutoff(oracle_mod, style, params, rc):
    r = rc * (1.0 - 1e-7)
    sf = _two(oracle_mod, r, style, params, rc, "force")
    es = _two(oracle_mod, r, style, params, rc, "energy")
    f_es = es.forces()[1, 0]
    assert abs(f_es) > 1e-6  # the unshifted force is finite at r_cut
    assert abs(sf.forces()[1, 0]) < 1e-5 * abs(f_es)
    assert abs(sf.energy()[0]) < 1e-12
    # beyond r_cut nothing interacts in either mode
    out = _two(oracle_mod, rc * 1.0000001, style, params, rc, "force")
    assert out.energy()[0] == 0.0 and np.all(out.forces() == 0.0)


@pytest.mark.parametrize("style,params,rc", FORMS)
def test_force_is_minus_energy_gradient(oracle_mod, style, params, rc):
    h = 1e-6
    for r in (0.85, 1.15, 1.9, rc - 0.05):
        up = _two(oracle_mod, r + h, style, params, rc).energy()[0]
        dn = _two(oracle_mod, r - h, style, params, rc).energy()[0]
        f = _two(oracle_mod, r, style, params, rc).forces()[1, 0]
        assert abs(f - (-(up - dn) / (2 * h))) < 1e-6 * max(1.0, abs(f))


def test_lj_values_at_two(oracle_mod):
    # closed forms at r = 2, r_cut = 2.5 (eps = sigma = 1): u(2) - u(2.5) = -0.045206546364,
    # F(2) = -0.181640625 (attractive), F(2.5) = -0.038999477453
    o = _two(oracle_mod, 2.0, "lj", (1.0, 1.0), 2.5)
    u_sf = -0.045206546364 + (2.0 - 2.5) * (-0.038999477453)
    f_sf = -0.181640625 - (-0.038999477453)
    assert abs(o.energy()[0] - u_sf) < 1e-11
    assert abs(o.forces()[1, 0] - f_sf) < 1e-11  # on the particle at x + r, along +x
    assert abs(o.forces()[0, 0] + f_sf) < 1e-11


@pytest.mark.parametrize("style,params,rc", FORMS)
def test_against_brute_force(oracle_mod, style, params, rc):
    rng = np.random.default_rng(7 + len(style))
    box = np.array([8.5, 9.0, 10.0])
    n = 260
    pos = rng.uniform(0, 1, (n, 3)) * box
    o = oracle_mod.OracleSystem(box, pos, np.zeros((n, 3)), np.zeros(n, np.int32), 1, [])
    o.set_pair_style(0, 0, style, params, rc)
    o.set_shift_mode("force")
    F, U, W = brute_fuw_style(box, pos, style, params, rc, shift_force=True)
    assert max_norm_rel(o.forces(), F) < 1e-12
    assert abs(o.energy()[0] - U) < 1e-12 * max(1.0, abs(U))
    assert max_norm_rel(o.virial(), W) < 1e-12


def test_mode_errors_and_default(oracle_mod):
    o = _two(oracle_mod, 1.2, "lj", (1.0, 1.0), 2.5, "energy")
    with pytest.raises(KeyError):
        o.set_shift_mode("smooth")
    assert o._lib.oracle_set_shift_mode(o._h, 2) != 0
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[1.0, 2.0, 3.0], [2.2, 2.0, 3.0]])
    d = oracle_mod.OracleSystem(box, pos, np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                                [(0, 0, 1.0, 1.0, 2.5)])
    assert d.energy()[0] == o.energy()[0]  # the default is the energy shift
