"""The continuous-batching request loop, on the CPU with a simulated executor and clock:
arrival-order admission by footprint and free slots, no overtaking at the queue head,
joining a running batch at block boundaries, budget and slot limits never exceeded,
latency bookkeeping, and the one-by-one baseline."""

import numpy as np
import pytest

from paper_1308_5587_amd import serve


class CapacityError(RuntimeError):
    code = -7


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)


class FakeSpec:
    def __init__(self, n):
        self.pos = np.zeros((n, 3))


class FakeBatch:
    """Executor with the batch interface: each block advances every resident replica by
    block_steps steps and costs time proportional to the resident atoms."""

    def __init__(self, clock, budget, slots, block_steps=10, sec_per_atom_step=1e-6):
        self.clock, self.budget, self.slots = clock, budget, slots
        self.block_steps, self.c = block_steps, sec_per_atom_step
        self.res = {}
        self.used = 0
        self.max_used = 0
        self.max_res = 0
        self.log = []

    def footprint(self, spec, nsteps=1):
        return spec.pos.shape[0] * 100

    def admit(self, spec, nsteps):
        fp = self.footprint(spec)
        free = [s for s in range(self.slots) if s not in self.res]
        if not free or self.used + fp > self.budget:
            raise CapacityError("full")
        s = free[0]
        self.res[s] = [spec.pos.shape[0], nsteps, 0, fp]
        self.used += fp
        self.max_used = max(self.max_used, self.used)
        self.max_res = max(self.max_res, len(self.res))
        self.log.append(("admit", s, self.clock.now()))
        return s

    def run_block(self):
        atoms = sum(v[0] for v in self.res.values() if v[2] < v[1])
        for v in self.res.values():
            v[2] = min(v[1], v[2] + self.block_steps)
        self.clock.t += atoms * self.block_steps * self.c

    def poll(self):
        return [s for s, v in self.res.items() if v[2] >= v[1]]

    def read(self, s):
        return {"steps": self.res[s][2]}

    def release(self, s):
        self.used -= self.res[s][3]
        del self.res[s]


def _reqs(spec_sizes, arrivals, steps):
    return [serve.Request(k, t, FakeSpec(n), s)
            for k, (n, t, s) in enumerate(zip(spec_sizes, arrivals, steps))]


def test_all_complete_within_limits():
    rng = np.random.default_rng(0)
    clock = SimClock()
    ex = FakeBatch(clock, budget=400_000, slots=4)
    n = rng.integers(100, 2000, size=40)
    t = np.cumsum(rng.exponential(0.05, size=40))
    st = rng.integers(10, 200, size=40)
    rep = serve.serve(ex, _reqs(n, t, st), clock=clock, keep_results=True)
    assert len(rep.requests) == 40
    assert ex.max_used <= 400_000 and ex.max_res <= 4
    for r in rep.requests:
        assert r.result["steps"] == r.nsteps
        assert r.arrival <= r.admitted <= r.finished
        # at least ceil(nsteps / block) blocks of its own atoms
        assert r.latency >= np.ceil(r.nsteps / 10) * 10 * r.n * 1e-6 - 1e-12
    s = rep.summary()
    assert s["requests"] == 40 and s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert s["atom_steps_per_s"] > 0


def test_arrival_order_and_no_overtaking():
    clock = SimClock()
    ex = FakeBatch(clock, budget=250_000, slots=8)
    # a big request arrives second and must wait for room; the small ones behind it wait too
    sizes = [2000, 2000, 100, 100, 100]
    rep = serve.serve(ex, _reqs(sizes, [0.0, 0.001, 0.002, 0.003, 0.004], [50] * 5), clock=clock)
    adm = {r.rid: r.admitted for r in rep.requests}
    assert adm[1] > adm[0]
    for k in (2, 3, 4):
        assert adm[k] >= adm[1]
    order = sorted(range(5), key=lambda k: (adm[k], k))
    assert order == [0, 1, 2, 3, 4]


def test_joins_running_batch_at_block_boundary():
    clock = SimClock()
    ex = FakeBatch(clock, budget=10**9, slots=4, block_steps=10)
    # the second request arrives while the first runs and is admitted before it finishes
    rep = serve.serve(ex, _reqs([1000, 1000], [0.0, 0.015], [100, 20]), clock=clock)
    a, b = rep.requests
    assert b.admitted < a.finished
    assert b.finished < a.finished
    # admitted at the first block boundary after its arrival (blocks of 0.01 s)
    assert abs(b.admitted - 0.02) < 1e-9


def test_request_that_never_fits_raises():
    clock = SimClock()
    ex = FakeBatch(clock, budget=1000, slots=2)
    with pytest.raises(CapacityError):
        serve.serve(ex, _reqs([100], [0.0], [10]), clock=clock)


def test_one_by_one_baseline():
    clock = SimClock()

    def run_alone(spec, nsteps):
        clock.t += spec.pos.shape[0] * nsteps * 1e-6
        return nsteps

    reqs = _reqs([1000, 500, 2000], [0.0, 0.01, 0.02], [100, 100, 100])
    rep = serve.serve_one_by_one(run_alone, reqs, clock=clock, keep_results=True)
    f = [r.finished for r in rep.requests]
    assert np.allclose(f, [0.1, 0.15, 0.35])
    assert [r.result for r in rep.requests] == [100, 100, 100]
    assert rep.summary()["p50_latency_s"] == pytest.approx(0.14)


class FailingBatch(FakeBatch):
    """Retires the replicas of the given request sizes with an error status (as the library
    does for a non-finite force); reading such a slot raises."""

    def __init__(self, *a, fail_sizes=(), **kw):
        super().__init__(*a, **kw)
        self.fail_sizes = set(fail_sizes)

    def slot_status(self, s):
        return -5 if self.res[s][0] in self.fail_sizes else 0

    def read(self, s):
        if self.slot_status(s):
            raise RuntimeError("read of a failed slot")
        return super().read(s)


def test_failed_requests_reported_apart():
    clock = SimClock()
    ex = FailingBatch(clock, budget=1_000_000, slots=3, fail_sizes={777})
    sizes = [500, 777, 600, 777, 900]
    rep = serve.serve(ex, _reqs(sizes, [0.0, 0.01, 0.02, 0.03, 0.04], [30, 30, 30, 30, 30]),
                      clock=clock, keep_results=True)
    assert [r.rid for r in rep.failed] == [1, 3]
    assert all(r.status == -5 and r.result is None for r in rep.failed)
    assert [r.rid for r in rep.requests] == [0, 2, 4]
    s = rep.summary()
    assert s["requests"] == 3 and s["failed"] == 2
    # throughput counts only the finished requests' work
    assert abs(s["atom_steps_per_s"] * s["wall_s"] - (500 + 600 + 900) * 30) < 1e-6
    assert ex.used == 0  # failed slots were released too
