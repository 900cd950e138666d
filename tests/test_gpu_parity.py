"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on identical
seeded inputs.

Bars: neighbour lists bit-exact as sorted tag-pair sets; FP64 forces, energies and virials
within 1e-10 max-norm relative; the mixed form within 1e-5 max-norm relative. Cases span
several cell tiles and ragged particle counts, boxes with fewer than three cells per axis, a
two-type mixture with per-pair cutoffs, and the full 1,048,576-particle fluid in the launch
configuration the benchmark uses."""

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen
from parity import (assert_full_list_equals_pairs, max_norm_rel, print_case, scalar_rel,
                    sort_pairs, unwrapped)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ljmd_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1308_5587_amd import ljmd

    ljmd.load()  # raises if the HIP library is missing
    return ljmd


def _pair(o_sys, g_sys, fp64=True, ff_tol=None):
    tol = ff_tol if ff_tol is not None else (1e-10 if fp64 else 1e-5)
    Fo = o_sys.forces()
    Fg = g_sys.forces()
    assert max_norm_rel(Fg, Fo) <= tol, max_norm_rel(Fg, Fo)
    Uo, Ko = o_sys.energy()
    Ug, Kg = g_sys.energy()
    assert scalar_rel(Ug, Uo) <= tol, (Ug, Uo)
    assert scalar_rel(Kg, Ko) <= 1e-12, (Kg, Ko)
    Wo = o_sys.virial()
    Wg = g_sys.virial()
    assert max_norm_rel(Wg, Wo) <= tol, (Wg, Wo)
    uo, wo = o_sys.per_particle()
    ug, wg = g_sys.per_particle()
    assert max_norm_rel(ug, uo) <= tol
    assert max_norm_rel(wg, wo) <= tol


def _list_parity(o_sys, g_sys, pos):
    po, xbo = o_sys.pairs()
    pg, xbg = g_sys.neighbor_pairs()
    assert np.array_equal(xbg, xbo)
    assert np.array_equal(xbg, pos)
    a = sort_pairs(po)
    b = sort_pairs(pg)
    assert a.shape == b.shape, (a.shape, b.shape)
    assert np.array_equal(a, b)
    # the full list the force kernel streams: both rows of every pair, nothing else
    counts, nb, xbf = g_sys.neighbor_list()
    assert np.array_equal(xbf, xbg)
    assert_full_list_equals_pairs(counts, nb, po)


def _step_past_rebuilds(g_sys, count=3, chunk=10, max_steps=400):
    """Step until the device has rebuilt the list at least `count` more times."""
    b0 = g_sys.stats()["rebuilds"]
    done = 0
    while g_sys.stats()["rebuilds"] < b0 + count:
        assert done < max_steps, "too few rebuilds"
        g_sys.step(chunk)
        done += chunk
    return done


def _rebuilt_list_parity(oracle_mod, g_sys, spec):
    """The list a device rebuild inside ljmd_step produced (from a drifted, cell-sorted
    state) against the oracle's list built at the same build positions."""
    counts, nb, xb = g_sys.neighbor_list()
    assert np.all(xb >= 0.0) and np.all(xb < spec.box[None, :])
    o = oracle_mod.OracleSystem(spec.box, xb, np.zeros_like(xb), spec.type, spec.ntypes,
                                spec.pairs)
    po, xbo = o.pairs()
    assert np.array_equal(xbo, xb)
    assert_full_list_equals_pairs(counts, nb, po)
    pg, _ = g_sys.neighbor_pairs()
    assert np.array_equal(sort_pairs(pg), sort_pairs(po))


@pytest.mark.parametrize("n,seed", [(4000, 1), (1, 3), (2, 4), (37, 5), (1001, 6), (6859, 7)])
def test_fp64_list_and_forces(ljmd_mod, oracle_mod, n, seed):
    print_case(f"fp64 list+forces n={n} seed={seed}")
    rho = 0.8442 if n >= 500 else 0.05
    s = gen.make_lj_fluid(n, rho=rho, T=1.2, seed=seed)
    if s.box[0] < 2 * 2.9:  # tiny counts: keep the box legal for r_cut + skin
        L = 6.0
        s = gen.LJSystemSpec(np.array([L] * 3), np.random.default_rng(seed).uniform(0, L, (n, 3)),
                             s.vel, s.type, 1, s.pairs)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    _list_parity(o, g, s.pos)
    _pair(o, g)


@pytest.mark.parametrize("n,rho", [(10000, 1.0), (8000, 1.0), (16000, 1.4)])
def test_dense_fluids_smaller_bricks(ljmd_mod, oracle_mod, n, rho):
    # 29, 37 and 47 atoms per cell: a 2 x 2 x 2 brick's 64-cell halo would not fit the LDS
    # tile, so bricks shrink to 2 x 2 x 1, 2 x 1 x 1 and single cells (48, 36, 27 halo cells)
    print_case(f"fp64 dense fluid n={n} rho={rho}")
    s = gen.make_lj_fluid(n, rho=rho, T=1.0, seed=21)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    _list_parity(o, g, s.pos)
    _pair(o, g)


def test_droplet_tiles_beyond_capacity(ljmd_mod, oracle_mod):
    # a dense block in a dilute vapour: the tile capacity is sized for the mean cell count
    # (about 7 atoms), so the bricks around the block (tiles of up to about 900 atoms) read
    # their neighbours from global memory in the list build and in the force kernels
    print_case("fp64 droplet: tiles beyond the LDS capacity")
    s = gen.make_lj_droplet(seed=5)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    _list_parity(o, g, s.pos)
    _pair(o, g)
    m = ljmd_mod.System.from_spec(s, precision="mixed")  # the fallback in FP32 pair arithmetic
    _pair(o, m, fp64=False)
    o.step(40)
    g.step(40)
    po, vo, io, _ = o.state()
    pg, vg, ig, _ = g.state()
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-9
    assert max_norm_rel(g.forces(), o.forces()) < 1e-9


def test_small_box_fewer_than_three_cells(ljmd_mod, oracle_mod):
    # L = 6.58 < 3 (r_cut + skin): two cells per axis, the stencil repeats cells
    print_case("fp64 small box 2 cells per axis")
    s = gen.make_lj_fluid(256, rho=256 / 6.58 ** 3, T=1.0, seed=11)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    g.step(0)  # lists and cells are set up lazily
    assert g.stats()["ncell"] == [2, 2, 2]
    _list_parity(o, g, s.pos)
    _pair(o, g)


def test_orthorhombic_box(ljmd_mod, oracle_mod):
    print_case("fp64 orthorhombic")
    rng = np.random.default_rng(12)
    box = np.array([9.0, 12.5, 17.25])
    n = 1500
    side = 12
    sites = np.stack(np.meshgrid(np.arange(side), np.arange(side), np.arange(side),
                                 indexing="ij"), -1).reshape(-1, 3)[:n]
    pos = (sites + 0.5) / side * box + rng.uniform(-0.05, 0.05, (n, 3))
    vel = rng.normal(0, 1, (n, 3))
    pairs = [(0, 0, 1.0, 0.7, 2.5)]
    o = oracle_mod.OracleSystem(box, pos, vel, np.zeros(n, np.int32), 1, pairs)
    g = ljmd_mod.System(box, pos, vel, np.zeros(n, np.int32), 1, pairs)
    _list_parity(o, g, pos)
    _pair(o, g)


def test_ka_mixture(ljmd_mod, oracle_mod):
    print_case("fp64 KA mixture n=8000")
    s = gen.make_ka_mixture(8000, seed=2)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    _list_parity(o, g, s.pos)
    _pair(o, g)


@pytest.mark.parametrize("tpp", [1, 2, 4, 8, 16])
def test_every_lane_count(ljmd_mod, oracle_mod, tpp):
    print_case(f"fp64 tpp={tpp}")
    s = gen.make_lj_fluid(3000, seed=21)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s, threads_per_particle=tpp, block_size=64 * (1 + tpp % 4))
    _list_parity(o, g, s.pos)
    _pair(o, g)


def test_frozen_tuning_table(ljmd_mod, oracle_mod, tmp_path):
    # a tuning table saved to JSON and loaded again fixes lanes and workgroup size of systems
    # in its key without timing runs; the tuner's own choices land in the table
    print_case("frozen tuning table")
    s = gen.make_lj_fluid(3000, seed=22)  # size bucket floor(log2 3000) = 11
    path = tmp_path / "tuning.json"
    ljmd_mod.set_tuning([dict(precision=0, multi_type=0, size_bucket=11,
                              threads_per_particle=8, block_size=192)])
    ljmd_mod.save_tuning(path)
    ljmd_mod.set_tuning([dict(precision=0, multi_type=0, size_bucket=11,
                              threads_per_particle=1, block_size=512)])
    ljmd_mod.load_tuning(path)
    g = ljmd_mod.System.from_spec(s, threads_per_particle=0, block_size=0)
    g.step(0)
    st = g.stats()
    assert (st["threads_per_particle"], st["block_size"]) == (8, 192)
    o = oracle_mod.OracleSystem.from_spec(s)
    _list_parity(o, g, s.pos)
    _pair(o, g)
    m = ljmd_mod.System.from_spec(gen.make_lj_fluid(5000, seed=23), precision="mixed")
    m.step(0)  # bucket 12, mixed: tuned, then recorded
    mst = m.stats()
    assert dict(precision=1, multi_type=0, size_bucket=12,
                threads_per_particle=mst["threads_per_particle"],
                block_size=mst["block_size"]) in ljmd_mod.tuning_table()


def test_mixed_forces(ljmd_mod, oracle_mod):
    print_case("mixed forces n=4000 and KA")
    s = gen.make_lj_fluid(4000, seed=1)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s, precision="mixed")
    _list_parity(o, g, s.pos)
    _pair(o, g, fp64=False)
    k = gen.make_ka_mixture(8000, seed=4)
    _pair(oracle_mod.OracleSystem.from_spec(k), ljmd_mod.System.from_spec(k, precision="mixed"),
          fp64=False)


def test_one_and_hundred_steps(ljmd_mod, oracle_mod):
    print_case("fp64 1 and 100 steps n=4000")
    s = gen.make_lj_fluid(4000, seed=1)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    o.step(1)
    g.step(1)
    po, vo, io, _ = o.state()
    pg, vg, ig, st = g.state()
    assert st == 1
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < 1e-12
    assert np.abs(vg - vo).max() < 1e-12
    _pair(o, g)
    o.step(99)
    g.step(99)
    po, vo, io, _ = o.state()
    pg, vg, ig, st = g.state()
    assert st == 100
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < 1e-8
    assert np.abs(vg - vo).max() < 1e-8
    assert max_norm_rel(g.forces(), o.forces()) < 1e-8
    assert g.stats()["rebuilds"] >= 5


@pytest.mark.parametrize("case,precision", [("fluid4000", "fp64"), ("fluid4000", "mixed"),
                                            ("box3cells", "fp64"), ("box2cells", "fp64"),
                                            ("ka8000", "mixed"), ("droplet", "fp64")])
def test_lists_after_device_rebuilds(ljmd_mod, oracle_mod, case, precision):
    """Lists rebuilt on the device inside ljmd_step (gated by the displacement check, from a
    drifted and cell-sorted state) are compared as full lists with the oracle's list at the
    same build positions, after at least three device rebuilds."""
    print_case(f"lists after device rebuilds: {case} {precision}")
    if case == "fluid4000":
        s = gen.make_lj_fluid(4000, seed=1)
    elif case == "box3cells":
        s = gen.make_lj_fluid(1000, rho=0.75, T=1.2, seed=31)
    elif case == "box2cells":
        s = gen.make_lj_fluid(256, rho=256 / 6.58 ** 3, T=1.0, seed=11)
    elif case == "ka8000":
        s = gen.make_ka_mixture(8000, seed=2)
    else:
        s = gen.make_lj_droplet(seed=5)
    g = ljmd_mod.System.from_spec(s, precision=precision)
    g.step(1)
    for chunk in (7, 11):
        _step_past_rebuilds(g, 3, chunk)
        _rebuilt_list_parity(oracle_mod, g, s)


@pytest.mark.parametrize("n,rho,box", [
    (1000, 0.75, None),                    # 3 cells per axis: z-layer bricks, whole-box halos
    (1320, None, (9.0, 12.5, 17.25)),      # 3, 4 and 5 cells: bricks one and two cells wide
    (1850, 0.8442, None),                  # 4 cells per axis: 2 x 1 x 1 bricks, halos span x
])
def test_hundred_steps_small_boxes(ljmd_mod, oracle_mod, n, rho, box):
    # small boxes: every brick's halo touches the periodic boundary, so the force kernel moves
    # staged atoms to their image nearest the brick centre on the axes where that is exact
    print_case(f"fp64 100 steps n={n} rho={rho} box={box}")
    if box is None:
        s = gen.make_lj_fluid(n, rho=rho, T=1.2, seed=31)
    else:
        rng = np.random.default_rng(32)
        b = np.array(box)
        side = np.array([8, 11, 15])  # lattice spacing 1.13 to 1.15 on every axis
        assert side.prod() == n
        sites = np.stack(np.meshgrid(*[np.arange(k) for k in side], indexing="ij"),
                         -1).reshape(-1, 3)
        pos = (sites + 0.5) / side * b + rng.uniform(-0.05, 0.05, (n, 3))
        s = gen.LJSystemSpec(b, pos, rng.normal(0, 1.1, (n, 3)), np.zeros(n, np.int32), 1,
                             [(0, 0, 1.0, 1.0, 2.5)])
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    for k in (1, 99):
        o.step(k)
        g.step(k)
        po, vo, io, _ = o.state()
        pg, vg, ig, _ = g.state()
        tol = 1e-12 if k == 1 else 1e-8
        assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < tol
        assert np.abs(vg - vo).max() < tol
        assert max_norm_rel(g.forces(), o.forces()) < (1e-10 if k == 1 else 1e-8)
    assert g.stats()["rebuilds"] >= 3


def test_mixed_steps_track_fp64(ljmd_mod, oracle_mod):
    print_case("mixed 1 and 100 steps")
    s = gen.make_lj_fluid(4000, seed=1)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s, precision="mixed")
    o.step(1)
    g.step(1)
    assert max_norm_rel(g.forces(), o.forces()) < 1e-5
    o.step(99)
    g.step(99)
    po, _, io, _ = o.state()
    pg, _, ig, _ = g.state()
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < 1e-3


def test_six_particle_parameter_sets(ljmd_mod):
    """The paper's pair-force unit-test recipe on the GPU path."""
    from sixparticle import calculator, load_fixture

    print_case("six particle")
    box, pos, params = load_fixture()
    g = ljmd_mod.System(box, pos, np.zeros((6, 3)), np.zeros(6, np.int32), 1,
                        [(0, 0, *params[0])])
    for (eps, sig, rc) in params:
        g.pair_lj_set(0, 0, eps, sig, rc)
        F, U, W, u_i, w_i = calculator(box, pos, eps, sig, rc)
        assert max_norm_rel(g.forces(), F) < 1e-12
        assert scalar_rel(g.energy()[0], U) < 1e-12
        assert max_norm_rel(g.virial(), W) < 1e-12
        ug, wg = g.per_particle()
        assert max_norm_rel(ug, u_i) < 1e-12 and max_norm_rel(wg, w_i) < 1e-12


def test_free_flight_and_images(ljmd_mod):
    print_case("free flight")
    rng = np.random.default_rng(4)
    n = 500
    box = np.array([7.0, 8.0, 9.0])
    pos = rng.uniform(0, 1, (n, 3)) * box
    vel = rng.normal(0, 30.0, (n, 3))
    g = ljmd_mod.System(box, pos, vel, np.zeros(n, np.int32), 1, [(0, 0, 0.0, 1.0, 2.5)])
    g.step(300)
    x, v, img, st = g.state()
    assert np.array_equal(v, vel)
    assert np.all(x >= 0) and np.all(x < box)
    assert np.abs(unwrapped(x, img, box) - (pos + 300 * 0.005 * vel)).max() < 1e-9
    assert np.abs(img).max() >= 1


def test_determinism_bitwise(ljmd_mod):
    print_case("determinism")
    s = gen.make_lj_fluid(20000, seed=8)
    a = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128)
    b = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128)
    a.step(200)
    b.step(200)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.forces(), b.forces())
    assert a.energy() == b.energy()


def test_graph_blocks_match_direct_launches(ljmd_mod):
    print_case("graph vs direct")
    s = gen.make_lj_fluid(5000, seed=9)
    a = ljmd_mod.System.from_spec(s, threads_per_particle=2, block_size=128, graph_steps=8)
    b = ljmd_mod.System.from_spec(s, threads_per_particle=2, block_size=128, graph_steps=-1)
    for k in (1, 17, 40, 2):
        a.step(k)
        b.step(k)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_overflow_recovery(ljmd_mod):
    print_case("overflow recovery")
    s = gen.make_lj_fluid(4000, seed=10)
    a = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128)
    b = ljmd_mod.System.from_spec(s, threads_per_particle=4, block_size=128, nlist_capacity=16)
    a.step(50)
    b.step(50)
    assert b.stats()["overflow_retries"] >= 1
    pa, va, ia, _ = a.state()
    pb, vb, ib, _ = b.state()
    assert np.abs(unwrapped(pa, ia, s.box) - unwrapped(pb, ib, s.box)).max() < 1e-10
    assert np.abs(va - vb).max() < 1e-10


def test_checkpoint_resume(ljmd_mod):
    print_case("checkpoint resume")
    s = gen.make_lj_fluid(3000, seed=13)
    a = ljmd_mod.System.from_spec(s)
    a.step(30)
    pos, vel, img, st = a.state()
    b = ljmd_mod.System.from_spec(s)
    b.set_state(pos, vel, img, st)
    a.set_state(pos, vel, img, st)  # same forced rebuild on both
    a.step(20)
    b.step(20)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_error_paths(ljmd_mod):
    print_case("error paths")
    E = ljmd_mod
    # box too small for r_cut + skin
    g = E.System(np.array([5.0] * 3), np.ones((2, 3)), np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                 [(0, 0, 1.0, 1.0, 2.5)])
    with pytest.raises(E.LjmdError) as e:
        g.step(1)
    assert e.value.code == E.LJMD_E_BOX
    # unset pair
    g = E.System(np.array([9.0] * 3), np.ones((2, 3)), np.zeros((2, 3)), np.array([0, 1], np.int32), 2,
                 [(0, 0, 1.0, 1.0, 2.5)])
    with pytest.raises(E.LjmdError) as e:
        g.forces()
    assert e.value.code == E.LJMD_E_STATE
    # overlap: non-finite force
    g = E.System(np.array([9.0] * 3), np.ones((2, 3)), np.zeros((2, 3)), np.zeros(2, np.int32), 1,
                 [(0, 0, 1.0, 1.0, 2.5)])
    with pytest.raises(E.LjmdError) as e:
        g.step(1)
    assert e.value.code == E.LJMD_E_NONFINITE


def test_full_size_fp64_and_mixed(ljmd_mod, oracle_mod):
    """N = 1,048,576 at density 0.8442 in the benchmark's launch configuration (autotuned
    lanes and workgroup, graph blocks): the whole list and all forces against the oracle."""
    print_case("full size N=1048576")
    s = gen.make_lj_fluid(1_048_576, rho=0.8442, T=1.2, seed=1)
    o = oracle_mod.OracleSystem.from_spec(s)
    g = ljmd_mod.System.from_spec(s)
    _list_parity(o, g, s.pos)
    assert max_norm_rel(g.forces(), o.forces()) <= 1e-10
    Uo, _ = o.energy()
    assert scalar_rel(g.energy()[0], Uo) <= 1e-10
    assert max_norm_rel(g.virial(), o.virial()) <= 1e-10
    m = ljmd_mod.System.from_spec(s, precision="mixed")
    assert max_norm_rel(m.forces(), o.forces()) <= 1e-5
    assert scalar_rel(m.energy()[0], Uo) <= 1e-5
    assert max_norm_rel(m.virial(), o.virial()) <= 1e-5
    uo, wo = o.per_particle()
    um, wm = m.per_particle()
    assert max_norm_rel(um, uo) <= 1e-5 and max_norm_rel(wm, wo) <= 1e-5
    ug, wg = g.per_particle()
    assert max_norm_rel(ug, uo) <= 1e-10 and max_norm_rel(wg, wo) <= 1e-10
    del uo, wo, um, wm, ug, wg
    # two steps on both paths
    o.step(2)
    g.step(2)
    assert max_norm_rel(g.forces(), o.forces()) <= 1e-10
    del o
    # lists rebuilt on the device during steps, against the oracle at their build positions
    _step_past_rebuilds(g, 3, 9)
    _rebuilt_list_parity(oracle_mod, g, s)


def test_full_size_ka_mixture(ljmd_mod, oracle_mod):
    """The Kob-Andersen mixture at its benchmark size (N = 262,144, density 1.2, per-pair
    cutoffs) in the launch configuration the library tunes for it: the whole list, and forces,
    energy and virial on the mixed path (the configuration's precision) and on the FP64 path,
    against the oracle; then ten steps of both paths."""
    print_case("full size KA mixture N=262144")
    s = gen.make_ka_mixture(262_144, seed=1)
    o = oracle_mod.OracleSystem.from_spec(s)
    m = ljmd_mod.System.from_spec(s, precision="mixed")
    _list_parity(o, m, s.pos)
    assert max_norm_rel(m.forces(), o.forces()) <= 1e-5
    Uo, _ = o.energy()
    assert scalar_rel(m.energy()[0], Uo) <= 1e-5
    assert max_norm_rel(m.virial(), o.virial()) <= 1e-5
    g = ljmd_mod.System.from_spec(s)
    assert max_norm_rel(g.forces(), o.forces()) <= 1e-10
    assert scalar_rel(g.energy()[0], Uo) <= 1e-10
    o.step(1)
    g.step(1)
    m.step(1)
    # one full step of the mixed path from the identical state
    assert max_norm_rel(m.forces(), o.forces()) <= 1e-5
    assert max_norm_rel(g.forces(), o.forces()) <= 1e-10
    o.step(9)
    g.step(9)
    m.step(9)
    assert max_norm_rel(g.forces(), o.forces()) <= 1e-10
    assert max_norm_rel(m.forces(), o.forces()) <= 1e-4
    po, _, io, _ = o.state()
    pg, _, ig, _ = g.state()
    assert np.abs(unwrapped(pg, ig, s.box) - unwrapped(po, io, s.box)).max() < 1e-10
    del o
    # lists rebuilt on the device during steps (mixed path), against the oracle
    _step_past_rebuilds(m, 3, 10)
    _rebuilt_list_parity(oracle_mod, m, s)
