"""Batched replicas on the GPU (ljmd_batch): every replica's result is the result it gets
when run alone, bit for bit, whatever else shares the batch and whenever it was admitted;
replica results also match the CPU FP64 oracle; slots and the memory budget are enforced.

Replica mixes are of uneven size and include a box with fewer than three cells per axis
and a two-type mixture (which switches every replica of the batch to the multi-type
kernels). Bitwise comparisons fix the lanes per particle, since the lane split orders the
force sums."""

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen
from parity import max_norm_rel, print_case, scalar_rel

pytestmark = pytest.mark.gpu

TPP, BLOCK = 4, 256


@pytest.fixture(scope="module")
def ljmd_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1308_5587_amd import ljmd

    ljmd.load()
    return ljmd


def _alone(ljmd, spec, nsteps, precision):
    g = ljmd.System.from_spec(spec, precision=precision, threads_per_particle=TPP,
                              block_size=BLOCK)
    g.step(nsteps)
    pos, vel, _, st = g.state()
    assert st == nsteps
    u, k = g.energy()
    return {"pos": pos, "vel": vel, "forces": g.forces(), "potential": u, "kinetic": k,
            "virial": g.virial()}


def _same(a, b):
    for key in ("pos", "vel", "forces", "virial"):
        assert np.array_equal(a[key], b[key]), key
    assert a["potential"] == b["potential"]
    assert a["kinetic"] == b["kinetic"]


def _mix():
    return [
        (gen.make_lj_fluid(300, rho=0.8, T=1.0, seed=11), 37),   # 2 cells per axis
        (gen.make_lj_fluid(1000, rho=0.6, T=1.4, seed=12), 50),
        (gen.make_lj_fluid(2500, rho=0.9, T=0.9, seed=13), 64),
        (gen.make_ka_mixture(1500, seed=14), 23),
    ]


def _run_until_done(batch, slots):
    pending = set(slots)
    blocks = 0
    while pending:
        batch.run_block()
        blocks += 1
        pending -= set(batch.poll())
        assert blocks < 1000
    return blocks


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(ljmd_mod, precision):
    print_case(f"batch of 4 uneven replicas vs alone, {precision}")
    mix = _mix()
    b = ljmd_mod.Batch(256 << 20, 8, precision=precision, block_steps=20,
                       threads_per_particle=TPP, block_size=BLOCK)
    slots = [b.admit(spec, n) for spec, n in mix]
    assert len(set(slots)) == 4
    _run_until_done(b, slots)
    for (spec, n), s in zip(mix, slots):
        assert b.slot_steps(s) == n
        _same(b.read(s), _alone(ljmd_mod, spec, n, precision))
    b.close()


@pytest.mark.parametrize("want_tpp,want_block", [(2, 0), (0, 0), (4, 0)])
def test_tuned_batch_equals_alone(ljmd_mod, want_tpp, want_block):
    # the first block tunes what is not given (workgroup size, or lanes and workgroup size);
    # the tuning trials rebuild the replicas' lists at their drifted positions, and the block
    # then retakes every replica's first half step from its state at t = 0, so each replica
    # still follows its alone run (with the lanes the batch settled on) bit for bit
    print_case(f"tuned batch (tpp={want_tpp}, block={want_block}) vs alone")
    mix = _mix()
    b = ljmd_mod.Batch(256 << 20, 8, precision="mixed", block_steps=20,
                       threads_per_particle=want_tpp, block_size=want_block)
    slots = [b.admit(spec, n) for spec, n in mix]
    _run_until_done(b, slots)
    st = b.stats()
    tpp, block = st["threads_per_particle"], st["block_size"]
    if want_tpp:
        assert tpp == want_tpp
    for (spec, n), s in zip(mix, slots):
        g = ljmd_mod.System.from_spec(spec, precision="mixed", threads_per_particle=tpp,
                                      block_size=block)
        g.step(n)
        pos, vel, _, _ = g.state()
        u, k = g.energy()
        _same(b.read(s), {"pos": pos, "vel": vel, "forces": g.forces(), "potential": u,
                          "kinetic": k, "virial": g.virial()})
    b.close()


def test_tile_overflow_decided_per_replica(ljmd_mod):
    # alone, the droplet's tile capacity is sized for its mean cell count and the bricks
    # around its dense block read neighbours from global memory. Beside a dense fluid the
    # batch's LDS allocation would hold those tiles, but the choice follows the replica's own
    # capacity, so the droplet takes the same path, and gets the same bits, in both runs.
    print_case("droplet beside a dense fluid: same force path alone and batched")
    mix = [(gen.make_lj_droplet(seed=6), 30), (gen.make_lj_fluid(4000, seed=7), 30)]
    b = ljmd_mod.Batch(256 << 20, 2, precision="fp64", block_steps=16,
                       threads_per_particle=TPP, block_size=BLOCK)
    slots = [b.admit(spec, n) for spec, n in mix]
    _run_until_done(b, slots)
    assert b.stats()["tile_capacity"] >= 1024
    for (spec, n), s in zip(mix, slots):
        _same(b.read(s), _alone(ljmd_mod, spec, n, "fp64"))
    b.close()


def test_admission_while_running(ljmd_mod):
    print_case("continuous admission: replicas join a running batch")
    mix = _mix()
    b = ljmd_mod.Batch(256 << 20, 4, precision="mixed", block_steps=10,
                       threads_per_particle=TPP, block_size=BLOCK)
    s0 = b.admit(*mix[0])
    s1 = b.admit(*mix[1])
    b.run_block()
    b.run_block()
    s2 = b.admit(*mix[2])  # joins after 20 steps of the others
    b.run_block()
    done = set(b.poll())
    s3 = b.admit(*mix[3])
    _run_until_done(b, [s0, s1, s2, s3])
    assert s0 not in done or b.slot_steps(s0) == mix[0][1]
    for (spec, n), s in zip(mix, [s0, s1, s2, s3]):
        _same(b.read(s), _alone(ljmd_mod, spec, n, "mixed"))
    # a released slot is reused and the new replica is again independent of the rest
    b.release(s1)
    s4 = b.admit(*mix[1])
    assert s4 == s1
    _run_until_done(b, [s4])
    _same(b.read(s4), _alone(ljmd_mod, mix[1][0], mix[1][1], "mixed"))
    b.close()


def test_batch_matches_oracle(ljmd_mod, oracle_mod):
    print_case("batched replicas vs oracle, fp64")
    mix = _mix()
    b = ljmd_mod.Batch(256 << 20, 4, precision="fp64", block_steps=20)
    slots = [b.admit(spec, n) for spec, n in mix]
    _run_until_done(b, slots)
    for (spec, n), s in zip(mix, slots):
        got = b.read(s)
        o = oracle_mod.OracleSystem.from_spec(spec)
        o.step(n)
        po, vo, _, _ = o.state()
        d = got["pos"] - po
        d -= spec.box[None, :] * np.rint(d / spec.box[None, :])
        assert np.abs(d).max() < 1e-8, np.abs(d).max()
        assert np.abs(got["vel"] - vo).max() < 1e-8
        assert max_norm_rel(got["forces"], o.forces()) < 1e-8
        uo, ko = o.energy()
        assert scalar_rel(got["potential"], uo) < 1e-9
        assert scalar_rel(got["kinetic"], ko) < 1e-9
    b.close()


def _compressing(n_side=12, rho=0.3, rate=1.0, seed=21):
    """A dilute lattice whose velocities point at the box centre: the list counts grow as it
    compresses, past the capacity sized at admission."""
    s = gen.make_lj_fluid(n_side ** 3, rho=rho, T=0.5, seed=seed)
    c = 0.5 * s.box[None, :]
    s.vel = np.ascontiguousarray(s.vel - rate * (s.pos - c))
    return s


def test_overflow_in_block_reruns_only_that_replica(ljmd_mod, oracle_mod):
    print_case("in-block list overflow: re-run of the overflowing replica only")
    comp = _compressing()
    # both start dilute, so the list capacity is sized for about 31 neighbours
    steady, n_steady = gen.make_lj_fluid(1000, rho=0.3, T=1.4, seed=12), 60
    b = ljmd_mod.Batch(256 << 20, 4, precision="fp64", block_steps=20,
                       threads_per_particle=TPP, block_size=BLOCK)
    sc = b.admit(comp, 60)
    ss = b.admit(steady, n_steady)
    cap0 = b.stats()["nlist_capacity"]
    _run_until_done(b, [sc, ss])
    st = b.stats()
    assert st["overflow_reruns"] >= 1 and st["nlist_capacity"] > cap0, (st, cap0)
    # the steady replica did not overflow: its result is untouched by the re-runs
    _same(b.read(ss), _alone(ljmd_mod, steady, n_steady, "fp64"))
    got = b.read(sc)
    o = oracle_mod.OracleSystem.from_spec(comp)
    o.step(60)
    po, vo, _, _ = o.state()
    d = got["pos"] - po
    d -= comp.box[None, :] * np.rint(d / comp.box[None, :])
    assert np.abs(d).max() < 1e-8
    assert np.abs(got["vel"] - vo).max() < 1e-8
    assert max_norm_rel(got["forces"], o.forces()) < 1e-8
    b.close()


def test_slots_budget_and_errors(ljmd_mod):
    print_case("batch capacity and error paths")
    E = ljmd_mod
    spec = gen.make_lj_fluid(500, seed=3)
    b = ljmd_mod.Batch(64 << 20, 2, precision="mixed", block_steps=10)
    fp = b.footprint(spec)
    assert fp > 500 * 200
    s0 = b.admit(spec, 5)
    s1 = b.admit(spec, 30)
    with pytest.raises(E.LjmdError) as e:
        b.admit(spec, 5)
    assert e.value.code == E.LJMD_E_CAPACITY
    with pytest.raises(E.LjmdError) as e:
        b.read(s1)  # still running
    assert e.value.code == E.LJMD_E_STATE
    b.run_block()
    assert b.poll() == [s0]
    assert b.slot_steps(s0) == 5 and b.slot_steps(s1) == 10
    b.release(s0)
    with pytest.raises(E.LjmdError) as e:
        b.read(s0)
    assert e.value.code == E.LJMD_E_STATE
    s2 = b.admit(spec, 4)
    assert s2 == s0
    _run_until_done(b, [s1, s2])
    st = b.stats()
    assert st["resident"] == 2 and st["running"] == 0 and st["used_bytes"] == 2 * fp
    # the whole box of 500 atoms is one staged tile (a capacity outside [64, 2560] would mean
    # every neighbour is read from global memory)
    assert 500 <= st["tile_capacity"] <= 2560, st
    # a box too small for the cutoff
    tiny = gen.make_lj_fluid(8, rho=0.8, seed=4)
    with pytest.raises(E.LjmdError) as e:
        b.footprint(tiny)
    assert e.value.code == E.LJMD_E_BOX
    b.close()
    # a budget that holds no replica of this size
    small = ljmd_mod.Batch(fp // 2 + 64 * 1024, 2, precision="mixed")
    with pytest.raises(E.LjmdError) as e:
        small.admit(spec, 5)
    assert e.value.code == E.LJMD_E_CAPACITY
    small.close()


def test_served_stream_results_equal_alone(ljmd_mod):
    print_case("served request stream: each result equals its alone run")
    from paper_1308_5587_amd import serve

    # arrivals far faster than service, so replicas share the GPU and queue for slots
    arrivals = gen.make_arrivals(6, rate=5000.0, seed=7, n_lo=512, n_hi=3000, steps_lo=100,
                                 steps_hi=300)
    mk = lambda p: gen.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)  # noqa: E731
    reqs = serve.requests_from_arrivals(arrivals, mk)
    b = ljmd_mod.Batch(128 << 20, 3, precision="mixed", block_steps=10,
                       threads_per_particle=TPP, block_size=BLOCK)
    rep = serve.serve(b, reqs, keep_results=True)
    b.close()
    assert len(rep.requests) == 6
    assert rep.peak_resident == 3, rep.peak_resident
    for r in rep.requests:
        _same(r.result, _alone(ljmd_mod, r.spec, r.nsteps, "mixed"))


def test_served_stream_matches_oracle_autotuned(ljmd_mod, oracle_mod):
    """A served stream on an autotuned batch (lanes and workgroup chosen at its first block):
    every request's result is checked against the FP64 oracle (one-step requests to the
    mixed single-step bar, longer ones to the mixed trajectory bound) and against its alone
    run with the lanes the batch settled on, bit for bit."""
    print_case("served autotuned stream vs oracle and vs alone")
    from paper_1308_5587_amd import serve

    arrivals = gen.make_arrivals(8, rate=5000.0, seed=9, n_lo=512, n_hi=4000, steps_lo=100,
                                 steps_hi=160)
    mk = lambda p: gen.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)  # noqa: E731
    reqs = serve.requests_from_arrivals(arrivals, mk)
    for r in reqs[::3]:
        r.nsteps = 1  # single-step requests: checked to the single-evaluation bar
    b = ljmd_mod.Batch(128 << 20, 3, precision="mixed", block_steps=10)
    rep = serve.serve(b, reqs, keep_results=True)
    st = b.stats()
    b.close()
    assert len(rep.requests) == 8 and not rep.failed
    assert rep.peak_resident == 3
    tpp, block = st["threads_per_particle"], st["block_size"]
    for r in rep.requests:
        got = r.result
        o = oracle_mod.OracleSystem.from_spec(r.spec)
        o.step(r.nsteps)
        po, vo, _, _ = o.state()
        d = got["pos"] - po
        d -= r.spec.box[None, :] * np.rint(d / r.spec.box[None, :])
        if r.nsteps == 1:
            assert max_norm_rel(got["forces"], o.forces()) <= 1e-5, r.rid
            assert np.abs(d).max() < 1e-7
        else:
            assert np.abs(d).max() < 1e-3, (r.rid, np.abs(d).max())
        uo, ko = o.energy()
        tol = 1e-5 if r.nsteps == 1 else 1e-3
        assert scalar_rel(got["potential"] + got["kinetic"], uo + ko) < tol, r.rid
        g = ljmd_mod.System.from_spec(r.spec, precision="mixed", threads_per_particle=tpp,
                                      block_size=block)
        g.step(r.nsteps)
        pos, vel, _, _ = g.state()
        u, k = g.energy()
        _same(got, {"pos": pos, "vel": vel, "forces": g.forces(), "potential": u,
                    "kinetic": k, "virial": g.virial()})


def test_full_size_batch_sampled_replicas(ljmd_mod, oracle_mod):
    """The benchmark's batch at full size: 512 replicas (N uniform in [256, 8192], density in
    [0.6, 0.9], T in [0.8, 1.5]), mixed precision, lanes and workgroup autotuned at the first
    block, one 100-step graph block. Sampled replicas equal their alone runs bit for bit (at
    the batch's lanes per particle) and track the FP64 oracle."""
    print_case("full batch: 512 replicas, one block; sampled replicas alone and vs oracle")
    params = gen.make_replica_specs(512, seed=0)
    specs = [gen.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed) for p in params]
    b = ljmd_mod.Batch(8 << 30, 512, precision="mixed", block_steps=100)
    slots = [b.admit(s, 100) for s in specs]
    b.run_block()
    assert set(b.poll()) == set(slots)
    st = b.stats()
    assert st["resident"] == 512 and st["running"] == 0
    tpp, block = st["threads_per_particle"], st["block_size"]
    for k in np.random.default_rng(5).choice(512, size=3, replace=False):
        spec = specs[k]
        got = b.read(slots[k])
        g = ljmd_mod.System.from_spec(spec, precision="mixed", threads_per_particle=tpp,
                                      block_size=block)
        g.step(100)
        pos, vel, _, _ = g.state()
        u, kin = g.energy()
        _same(got, {"pos": pos, "vel": vel, "forces": g.forces(), "potential": u,
                    "kinetic": kin, "virial": g.virial()})
        o = oracle_mod.OracleSystem.from_spec(spec)
        o.step(100)
        po, _, _, _ = o.state()
        d = got["pos"] - po
        d -= spec.box[None, :] * np.rint(d / spec.box[None, :])
        assert np.abs(d).max() < 1e-3, (k, np.abs(d).max())
    b.close()
