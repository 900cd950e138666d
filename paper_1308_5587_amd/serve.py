"""Continuous-batching request loop for LJ replica runs.

Requests (a replica's initial condition and a number of NVE steps) arrive over time. The
loop admits waiting requests in arrival order whenever a slot and enough of the device
memory budget are free (the footprint the batch library reports), advances every resident
replica by one block of steps per iteration, and retires replicas as they finish, so work
that arrives while other replicas are on the GPU joins them at the next block boundary.
Replica state stays on the device from admission to retirement.

The executor is anything with the batch interface of ``ljmd.Batch`` (footprint, admit,
run_block, poll, read, release, and optionally slot_status); the scheduling logic here
holds no simulation arithmetic. Latency of a request is its completion time minus its
arrival time on the loop's clock. A request whose replica the executor retired with an
error (slot_status non-zero) is reported as failed: it is neither read nor counted in the
latency and throughput figures.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

CAPACITY_CODE = -7  # LJMD_E_CAPACITY


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    spec: object            # LJSystemSpec-like: box, pos, vel, type, ntypes, pairs
    nsteps: int
    admitted: float = -1.0
    finished: float = -1.0
    slot: int = -1
    status: int = 0         # 0, or the error code the replica was retired with
    refused: int = 0        # admissions refused for capacity (no slot or budget) while at the head
    result: dict = field(default=None, repr=False)

    @property
    def n(self):
        return int(np.asarray(self.spec.pos).shape[0])

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class ServeReport:
    requests: list          # finished requests, by id
    wall_s: float
    blocks: int
    peak_resident: int
    failed: list = field(default_factory=list)  # requests retired with an error

    def latencies(self):
        return np.array([r.latency for r in self.requests], dtype=np.float64)

    def summary(self):
        lat = self.latencies()
        work = float(sum(r.n * r.nsteps for r in self.requests))
        return {
            "requests": len(self.requests),
            "wall_s": self.wall_s,
            "atom_steps_per_s": work / self.wall_s if self.wall_s > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else 0.0,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else 0.0,
            "mean_latency_s": float(lat.mean()) if len(lat) else 0.0,
            "blocks": self.blocks,
            "peak_resident": self.peak_resident,
            "failed": len(self.failed),
            "refused_for_capacity": sum(1 for r in self.requests if r.refused),
        }


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def wait_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


def _is_capacity(err):
    return getattr(err, "code", None) == CAPACITY_CODE


def serve(executor, requests, clock=None, keep_results=False, max_blocks=10_000_000):
    """Run ``requests`` (sorted or not by arrival) through ``executor`` with continuous
    batching. Returns a ServeReport; each request gets admitted/finished times (and its
    result when keep_results)."""
    clock = clock or WallClock()
    incoming = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    waiting: deque = deque()
    resident = {}
    blocks = 0
    peak = 0
    done = []
    failed = []
    slot_status = getattr(executor, "slot_status", None)
    while incoming or waiting or resident:
        now = clock.now()
        while incoming and incoming[0].arrival <= now:
            waiting.append(incoming.popleft())
        # admit in arrival order; the head of the queue waits for room (no overtaking, so a
        # large request is never starved by a stream of small ones)
        while waiting:
            r = waiting[0]
            try:
                slot = executor.admit(r.spec, r.nsteps)
            except Exception as e:  # noqa: BLE001 - only the capacity code is expected
                if _is_capacity(e) and resident:
                    r.refused += 1
                    break
                raise
            waiting.popleft()
            r.slot = slot
            r.admitted = clock.now()
            resident[slot] = r
        peak = max(peak, len(resident))
        if not resident:
            if incoming:
                clock.wait_until(incoming[0].arrival)
            continue
        executor.run_block()
        blocks += 1
        if blocks > max_blocks:
            raise RuntimeError("serve loop exceeded its block limit")
        for slot in executor.poll():
            r = resident.pop(slot, None)
            if r is None:
                continue
            r.finished = clock.now()
            r.status = int(slot_status(slot)) if slot_status else 0
            if r.status != 0:
                executor.release(slot)
                failed.append(r)
                continue
            if keep_results:
                r.result = executor.read(slot)
            executor.release(slot)
            done.append(r)
    wall = clock.now()
    done.sort(key=lambda r: r.rid)
    failed.sort(key=lambda r: r.rid)
    return ServeReport(done, wall, blocks, peak, failed)


def serve_one_by_one(run_alone, requests, clock=None, keep_results=False):
    """The same request stream served one request at a time: ``run_alone(spec, nsteps)``
    runs a replica to completion and returns its result. Requests queue in arrival order."""
    clock = clock or WallClock()
    done = []
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        clock.wait_until(r.arrival)
        r.admitted = clock.now()
        res = run_alone(r.spec, r.nsteps)
        r.finished = clock.now()
        if keep_results:
            r.result = res
        done.append(r)
    wall = clock.now()
    done.sort(key=lambda r: r.rid)
    return ServeReport(done, wall, 0, 1)


def requests_from_arrivals(arrivals, make_spec):
    """Requests from (arrival_time, ReplicaParams) pairs; ``make_spec(params)`` builds the
    initial condition of each."""
    return [Request(k, float(t), make_spec(p), int(p.steps)) for k, (t, p) in enumerate(arrivals)]
