"""Pins of the oracle's other pair forms (Mie, Gaussian, Yukawa, and WCA as the LJ form cut
at 2^(1/6) sigma; the paper lists them among its pair potentials, Section "Capabilities"):
closed forms, the Mie form's reduction to LJ at (12, 6), F = -du/dr by central difference,
Newton's third law, and an independent numpy brute force on random boxes."""

import math

import numpy as np
import pytest

from brute import brute_fuw_style
from parity import max_norm_rel

FORMS = [("mie", (1.3, 1.1, 14.0, 7.0), 2.8), ("gauss", (2.0, 0.9, 0.0, 0.0), 2.7),
         ("yukawa", (1.5, 0.8, 0.0, 0.0), 2.6)]


def _two(oracle_mod, r, style, params, rc, L=10.0):
    box = np.array([L, L, L])
    pos = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
    o = oracle_mod.OracleSystem(box, pos, np.zeros((2, 3)), np.zeros(2, np.int32), 1, [])
    o.set_pair_style(0, 0, style, params, rc)
    return o


def test_mie_12_6_is_lj(oracle_mod):
    rng = np.random.default_rng(1)
    box = np.array([9.0, 9.0, 9.0])
    pos = rng.uniform(0, 9.0, (300, 3))
    a = oracle_mod.OracleSystem(box, pos, np.zeros((300, 3)), np.zeros(300, np.int32), 1,
                                [(0, 0, 1.2, 0.5, 2.5)])
    b = oracle_mod.OracleSystem(box, pos, np.zeros((300, 3)), np.zeros(300, np.int32), 1, [])
    b.set_pair_style(0, 0, "mie", (1.2, 0.5, 12.0, 6.0), 2.5)
    assert max_norm_rel(b.forces(), a.forces()) < 1e-13
    assert abs(b.energy()[0] - a.energy()[0]) < 1e-13 * abs(a.energy()[0])


def test_gaussian_closed_form(oracle_mod):
    eps, sig, rc = 2.0, 0.9, 2.7
    for r in (0.45, 0.9, 1.7):
        o = _two(oracle_mod, r, "gauss", (eps, sig), rc)
        u_ref = eps * math.exp(-r * r / (2 * sig * sig)) - eps * math.exp(-rc * rc / (2 * sig * sig))
        f_ref = eps * r / (sig * sig) * math.exp(-r * r / (2 * sig * sig))  # repulsive
        U, _ = o.energy()
        F = o.forces()
        assert abs(U - u_ref) < 1e-14
        assert abs(F[0, 0] + f_ref) < 1e-13 and abs(F[1, 0] - f_ref) < 1e-13
        assert abs(o.virial()[0] - r * f_ref) < 1e-13


def test_yukawa_closed_form(oracle_mod):
    eps, kappa, rc = 1.5, 0.8, 2.6
    for r in (0.7, 1.0, 2.2):
        o = _two(oracle_mod, r, "yukawa", (eps, kappa), rc)
        u_ref = eps * math.exp(-kappa * r) / r - eps * math.exp(-kappa * rc) / rc
        f_ref = eps * math.exp(-kappa * r) * (1 + kappa * r) / (r * r)
        U, _ = o.energy()
        F = o.forces()
        assert abs(U - u_ref) < 1e-14
        assert abs(F[1, 0] - f_ref) < 1e-13 and abs(F[0, 0] + f_ref) < 1e-13


def test_wca_is_lj_cut_at_minimum(oracle_mod):
    rc = 2.0 ** (1.0 / 6.0)
    box = np.array([10.0] * 3)
    for r, u_ref in ((1.0, 1.0), (rc * 0.999999, None)):
        pos = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]])
        o = oracle_mod.OracleSystem(box, pos, np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                                    [(0, 0, 1.0, 1.0, rc)])
        U, _ = o.energy()
        if u_ref is not None:
            assert abs(U - u_ref) < 1e-14  # 4(1 - 1) + eps
        else:
            assert 0.0 <= U < 1e-9 and np.abs(o.forces()).max() < 1e-4


@pytest.mark.parametrize("style,params,rc", FORMS)
def test_force_is_minus_energy_gradient(oracle_mod, style, params, rc):
    h = 1e-6
    for r in (0.8, 1.1, 1.9):
        up = _two(oracle_mod, r + h, style, params, rc).energy()[0]
        dn = _two(oracle_mod, r - h, style, params, rc).energy()[0]
        f = _two(oracle_mod, r, style, params, rc).forces()[1, 0]
        assert abs(f - (-(up - dn) / (2 * h))) < 1e-6 * max(1.0, abs(f))


@pytest.mark.parametrize("style,params,rc", FORMS)
def test_forms_against_brute_force(oracle_mod, style, params, rc):
    rng = np.random.default_rng(hash(style) % 1000)
    box = np.array([8.5, 9.0, 10.0])
    n = 260
    pos = rng.uniform(0, 1, (n, 3)) * box
    o = oracle_mod.OracleSystem(box, pos, np.zeros((n, 3)), np.zeros(n, np.int32), 1, [])
    o.set_pair_style(0, 0, style, params, rc)
    F, U, W = brute_fuw_style(box, pos, style, params, rc)
    assert max_norm_rel(o.forces(), F) < 1e-12
    assert abs(o.energy()[0] - U) < 1e-12 * max(1.0, abs(U))
    assert max_norm_rel(o.virial(), W) < 1e-12
    assert np.abs(o.forces().sum(0)).max() < 1e-10 * np.abs(F).max()


def test_style_argument_errors(oracle_mod):
    o = _two(oracle_mod, 1.0, "gauss", (1.0, 1.0), 2.5)
    for style, params in (("mie", (1.0, 1.0, 6.0, 12.0)), ("mie", (1.0, 0.0, 12.0, 6.0)),
                          ("gauss", (1.0, 0.0)), ("yukawa", (1.0, -1.0))):
        with pytest.raises(oracle_mod.OracleError):
            o.set_pair_style(0, 0, style, params, 2.5)
