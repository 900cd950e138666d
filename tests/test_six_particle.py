"""The paper's LJ unit-test recipe (Section "Software engineering", Testing) against the
CPU oracle: six particles, some pairs through the periodic boundaries, the parameters changed
on the same system between evaluations, force, energy and virial checked every time."""

import numpy as np

from sixparticle import calculator, load_fixture


def test_fixture_geometry():
    box, pos, params = load_fixture()
    assert pos.shape == (6, 3) and len(params) == 3
    assert np.all(pos >= 0) and np.all(pos < box)


def test_oracle_six_particle(oracle_mod):
    box, pos, params = load_fixture()
    o = oracle_mod.OracleSystem(box, pos, np.zeros((6, 3)), np.zeros(6, np.int32), 1,
                                [(0, 0, *params[0])])
    for (eps, sig, rc) in params:
        o.set_pair(0, 0, eps, sig, rc)
        F, U, W, u_i, w_i = calculator(box, pos, eps, sig, rc)
        Fo = o.forces()
        Uo, _ = o.energy()
        uo, wo = o.per_particle()
        scale = np.abs(F).max()
        assert np.abs(Fo - F).max() <= 1e-12 * scale
        assert abs(Uo - U) <= 1e-12 * max(1.0, abs(U))
        assert np.abs(o.virial() - W).max() <= 1e-12 * np.abs(W).max()
        assert np.abs(uo - u_i).max() <= 1e-12 * np.abs(u_i).max()
        assert np.abs(wo - w_i).max() <= 1e-12 * np.abs(w_i).max()
    # the third parameter set (r_cut = 1.3) keeps only the short pairs 0-1, 0-2, 3-4
    assert np.abs(F[5]).max() == 0.0
