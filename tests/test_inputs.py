"""Seeded input generators: sizes, densities, temperatures and determinism."""

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen


@pytest.mark.parametrize("n", [1, 2, 27, 1000, 4000, 5000])
def test_fluid_shape_density_temperature(n):
    s = gen.make_lj_fluid(n, rho=0.8442, T=1.2, seed=1)
    L = s.box[0]
    assert s.pos.shape == (n, 3) and s.vel.shape == (n, 3) and s.type.shape == (n,)
    assert np.isclose(n / L ** 3, 0.8442, rtol=1e-13)
    assert np.all(s.pos >= 0) and np.all(s.pos < L)
    if n > 1:
        p = s.vel.sum(axis=0)
        assert np.all(np.abs(p) < 1e-10)
        T = np.sum(s.vel ** 2) / (3 * n - 3)
        assert abs(T - 1.2) < 1e-12


def test_lattice_sites_distinct_and_vacancies():
    s = gen.make_lj_fluid(4000, seed=1, jitter=0.0)
    side = gen.cube_side(4000)
    assert side == 16
    a = s.box[0] / side
    idx = np.rint(s.pos / a - 0.5).astype(int)
    flat = (idx[:, 0] * side + idx[:, 1]) * side + idx[:, 2]
    assert len(np.unique(flat)) == 4000
    assert np.all(np.diff(flat) > 0)  # chosen sites sorted ascending


def test_cube_side_exact():
    assert gen.cube_side(1) == 1
    assert gen.cube_side(8) == 2
    assert gen.cube_side(9) == 3
    assert gen.cube_side(1_048_576) == 102
    assert gen.cube_side(262_144) == 64


def test_seed_determinism():
    a = gen.make_lj_fluid(500, seed=7)
    b = gen.make_lj_fluid(500, seed=7)
    c = gen.make_lj_fluid(500, seed=8)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    assert not np.array_equal(a.pos, c.pos)


def test_ka_counts():
    s = gen.make_ka_mixture(262_144)
    assert s.ntypes == 2
    assert int(np.sum(s.type == 0)) == 209_715
    assert int(np.sum(s.type == 1)) == 52_429
    assert np.isclose(s.box[0], 60.2257, atol=1e-3)
    tab = {(a, b): (e, sg, rc) for (a, b, e, sg, rc) in s.pairs}
    assert tab[(0, 1)] == (1.5, 0.8, 2.0)
    assert np.isclose(tab[(1, 1)][2], 2.2)


def test_replica_and_arrival_streams():
    reps = gen.make_replica_specs(512, seed=0)
    ns = np.array([r.n for r in reps])
    assert ns.min() >= 256 and ns.max() <= 8192
    assert 1.9e6 < ns.sum() < 2.4e6
    arr = gen.make_arrivals(1000, rate=10.0, seed=2)
    t = np.array([a[0] for a in arr])
    assert np.all(np.diff(t) >= 0)
    nn = np.array([a[1].n for a in arr])
    st = np.array([a[1].steps for a in arr])
    assert nn.min() >= 512 and nn.max() <= 65536
    assert st.min() >= 1000 and st.max() <= 10000
    # mean of a log-uniform on [512, 65536] is (65536 - 512) / ln(128) ~ 13401
    assert 11000 < nn.mean() < 16000
