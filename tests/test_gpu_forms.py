"""Other pair forms on the GPU (ljmd_pair_set: Mie, Gaussian, Yukawa, WCA) through the C ABI,
against the CPU FP64 oracle on identical seeded inputs: lists bit-exact as full lists, FP64
forces, energy and virial within 1e-10, the mixed form within 1e-5, 30 steps within 1e-9;
one and two types (the multi-type kernels)."""

import math

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen
from parity import (assert_full_list_equals_pairs, max_norm_rel, print_case, scalar_rel,
                    unwrapped)

pytestmark = pytest.mark.gpu

FORMS = [("mie", (1.0, 1.0, 14.0, 7.0), 2.5), ("gauss", (3.0, 1.0), 2.8),
         ("yukawa", (2.0, 1.2), 2.6), ("wca", (1.0, 1.0), 0.0)]


@pytest.fixture(scope="module")
def ljmd_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1308_5587_amd import ljmd

    ljmd.load()
    return ljmd


def _oracle_pair(o, a, b, form, params, rc):
    if form == "wca":
        o.set_pair(a, b, params[0], params[1], 2.0 ** (1.0 / 6.0) * params[1])
    else:
        o.set_pair_style(a, b, form, params, rc)


def _check(o, g, tol):
    assert max_norm_rel(g.forces(), o.forces()) <= tol
    Uo, Ko = o.energy()
    Ug, Kg = g.energy()
    assert scalar_rel(Ug, Uo) <= tol, (Ug, Uo)
    assert max_norm_rel(g.virial(), o.virial()) <= tol
    uo, wo = o.per_particle()
    ug, wg = g.per_particle()
    assert max_norm_rel(ug, uo) <= tol and max_norm_rel(wg, wo) <= tol


@pytest.mark.parametrize("form,params,rc", FORMS)
def test_form_single_type(ljmd_mod, oracle_mod, form, params, rc):
    print_case(f"pair form {form}")
    s = gen.make_lj_fluid(4000, rho=0.8442 if form != "gauss" else 0.5, T=1.2, seed=3)
    o = oracle_mod.OracleSystem(s.box, s.pos, s.vel, s.type, 1, [])
    _oracle_pair(o, 0, 0, form, params, rc)
    g = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 1, [])
    g.pair_set(0, 0, form, params, rc)
    po, _ = o.pairs()
    counts, nb, xb = g.neighbor_list()
    assert np.array_equal(xb, s.pos)
    assert_full_list_equals_pairs(counts, nb, po)
    _check(o, g, 1e-10)
    m = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 1, [], precision="mixed")
    m.pair_set(0, 0, form, params, rc)
    _check(o, m, 1e-5)
    o.step(30)
    g.step(30)
    po_, vo, io, _ = o.state()
    pg, vg, ig, _ = g.state()
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po_, io, s.box)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-9


def test_form_two_types(ljmd_mod, oracle_mod):
    print_case("pair form mie, two types with per-pair parameters")
    s = gen.make_ka_mixture(6000, seed=5)
    table = {(0, 0): (1.0, 1.0, 12.0, 6.0), (0, 1): (1.5, 0.8, 13.0, 6.5),
             (1, 1): (0.5, 0.88, 11.0, 5.5)}
    o = oracle_mod.OracleSystem(s.box, s.pos, s.vel, s.type, 2, [])
    g = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 2, [])
    for (a, b), p in table.items():
        o.set_pair_style(a, b, "mie", p, 2.5 * p[1])
        g.pair_set(a, b, "mie", p, 2.5 * p[1])
    po, _ = o.pairs()
    counts, nb, _ = g.neighbor_list()
    assert_full_list_equals_pairs(counts, nb, po)
    _check(o, g, 1e-10)
    o.step(20)
    g.step(20)
    assert max_norm_rel(g.forces(), o.forces()) < 1e-9


def test_one_form_per_system(ljmd_mod):
    print_case("pair forms: a second form in one system is refused")
    s = gen.make_ka_mixture(500, seed=6)
    g = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 2, [])
    g.pair_set(0, 0, "gauss", (1.0, 1.0), 2.5)
    with pytest.raises(ljmd_mod.LjmdError) as e:
        g.pair_set(0, 1, "yukawa", (1.0, 1.0), 2.5)
    assert e.value.code == ljmd_mod.LJMD_E_INVAL
    g.pair_set(0, 0, "yukawa", (1.0, 1.0), 2.5)  # replacing the only set pair is allowed
    with pytest.raises(ljmd_mod.LjmdError):
        g.pair_set(1, 1, "mie", (1.0, 1.0, 6.0, 12.0), 2.5)  # n <= m
    with pytest.raises(ljmd_mod.LjmdError):
        g.pair_set(1, 1, "wca", (1.0, 1.0), 2.5)  # WCA takes its own cut


SF_FORMS = [("lj", (1.0, 1.0), 2.5), ("mie", (1.0, 1.0, 14.0, 7.0), 2.5),
            ("gauss", (3.0, 1.0), 2.8), ("yukawa", (2.0, 1.2), 2.6)]


@pytest.mark.parametrize("form,params,rc", SF_FORMS)
def test_shifted_force(ljmd_mod, oracle_mod, form, params, rc):
    print_case(f"shifted force, pair form {form}")
    s = gen.make_lj_fluid(4000, rho=0.8442 if form != "gauss" else 0.5, T=1.2, seed=4)
    o = oracle_mod.OracleSystem(s.box, s.pos, s.vel, s.type, 1, [])
    o.set_pair_style(0, 0, form, params, rc)
    o.set_shift_mode("force")
    g = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 1, [])
    g.pair_set(0, 0, form, params, rc)
    g.set_pair_shift("force")
    _check(o, g, 1e-10)
    m = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 1, [], precision="mixed")
    m.pair_set(0, 0, form, params, rc)
    m.set_pair_shift("force")
    _check(o, m, 1e-5)
    o.step(30)
    g.step(30)
    po_, vo, io, _ = o.state()
    pg, vg, ig, _ = g.state()
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po_, io, s.box)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-9
    _check(o, g, 1e-8)
    # back to the energy shift: the plain form again
    g.set_pair_shift("energy")
    o.set_shift_mode("energy")
    _check(o, g, 1e-10)


def test_shifted_force_errors(ljmd_mod):
    print_case("shifted force: unknown mode, tree lists refused")
    s = gen.make_lj_fluid(500, rho=0.8, T=1.0, seed=2)
    g = ljmd_mod.System(s.box, s.pos, s.vel, s.type, 1, [(0, 0, 1.0, 1.0, 2.5)])
    with pytest.raises(ljmd_mod.LjmdError) as e:
        ljmd_mod._check(g._lib.ljmd_set_pair_shift(g._h, 2))
    assert e.value.code == ljmd_mod.LJMD_E_INVAL
    with pytest.raises(KeyError):
        g.set_pair_shift("smooth")
    g.set_pair_shift("force")
    g.set_nlist("tree")
    with pytest.raises(ljmd_mod.LjmdError) as e:
        g.step(1)
    assert e.value.code == ljmd_mod.LJMD_E_INVAL
