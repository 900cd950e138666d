"""Seeded synthetic inputs for Lennard-Jones systems.

This module builds initial conditions only: lattice sites, jitter, Maxwell-Boltzmann
velocities, type assignments, replica parameter sets and request arrival streams. It holds
none of the simulation arithmetic (no distances, forces or integration), so both the GPU
library and the CPU oracle may be fed from it.

The recipes follow the user-level setup of the paper's molecular-dynamics example
(Section "Capabilities", Molecular dynamics listing: a simple-cubic lattice, randomized
velocities at kT = 1.2 from a seed) and the Lennard-Jones liquid benchmark state point
(Section "Performance"). Where the paper is silent the readings are:

* N not a perfect cube: ``n_side = ceil(N ** (1/3))`` sites per axis at spacing
  ``a = L / n_side``; N of the ``n_side**3`` sites are chosen by a seeded permutation and
  sorted ascending; site centres at ``(index + 1/2) * a``.
* Jitter: uniform in ``[-jitter, +jitter)`` per component.
* Velocities: normal with variance ``T / m`` per component, mean subtracted, rescaled so
  that the kinetic temperature with ``3N - 3`` degrees of freedom equals ``T`` exactly.
* Draw order from one ``numpy.random.default_rng(seed)``: sites, jitter, velocities, types.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "LJSystemSpec",
    "make_lj_fluid",
    "make_ka_mixture",
    "ka_pair_table",
    "lj_single_pair_table",
    "make_replica_specs",
    "make_lj_droplet",
    "make_arrivals",
    "cube_side",
]


@dataclass
class LJSystemSpec:
    """Host-side initial condition of one LJ system (float64, tag order)."""

    box: np.ndarray  # (3,) float64 box edges
    pos: np.ndarray  # (N, 3) float64, inside [0, L)
    vel: np.ndarray  # (N, 3) float64
    type: np.ndarray  # (N,) int32
    ntypes: int
    # pair table: list of (a, b, epsilon, sigma, r_cut)
    pairs: list = field(default_factory=list)
    seed: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def cube_side(n: int) -> int:
    """Smallest integer s with s**3 >= n (exact integer arithmetic)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    s = max(1, int(round(n ** (1.0 / 3.0))))
    while s ** 3 < n:
        s += 1
    while s > 1 and (s - 1) ** 3 >= n:
        s -= 1
    return s


def _lattice_positions(rng, n: int, L: float, jitter: float) -> np.ndarray:
    side = cube_side(n)
    a = L / side
    if 0.5 * a <= jitter:
        raise ValueError("lattice spacing too small for the requested jitter")
    total = side ** 3
    if total == n:
        chosen = np.arange(n, dtype=np.int64)
        # keep the draw sequence identical whether or not vacancies exist
        rng.permutation(total)
    else:
        chosen = np.sort(rng.permutation(total)[:n]).astype(np.int64)
    ix = chosen // (side * side)
    iy = (chosen // side) % side
    iz = chosen % side
    sites = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    pos = (sites + 0.5) * a
    pos += rng.uniform(-jitter, jitter, size=(n, 3))
    # sites at (i + 1/2) a with |jitter| < a/2 stay strictly inside [0, L)
    assert np.all(pos >= 0.0) and np.all(pos < L)
    return pos


def _mb_velocities(rng, n: int, T: float, mass: float = 1.0) -> np.ndarray:
    vel = rng.normal(0.0, math.sqrt(T / mass), size=(n, 3))
    if n > 1:
        vel -= vel.mean(axis=0, keepdims=True)
        dof = 3 * n - 3
        kin = 0.5 * mass * float(np.sum(vel * vel))
        t_now = 2.0 * kin / dof
        if t_now > 0.0:
            vel *= math.sqrt(T / t_now)
    else:
        vel[:] = 0.0
    return vel


def lj_single_pair_table(r_cut: float = 2.5, epsilon: float = 1.0, sigma: float = 1.0):
    return [(0, 0, epsilon, sigma, r_cut)]


def make_lj_fluid(
    n: int,
    rho: float = 0.8442,
    T: float = 1.2,
    seed: int = 1,
    jitter: float = 0.05,
    r_cut: float = 2.5,
) -> LJSystemSpec:
    """Single-type LJ fluid: cubic box at number density ``rho``, simple-cubic lattice
    plus uniform jitter, Maxwell-Boltzmann velocities at ``T`` with zero net momentum."""
    rng = np.random.default_rng(seed)
    L = (n / rho) ** (1.0 / 3.0)
    pos = _lattice_positions(rng, n, L, jitter)
    vel = _mb_velocities(rng, n, T)
    typ = np.zeros(n, dtype=np.int32)
    return LJSystemSpec(
        box=np.array([L, L, L], dtype=np.float64),
        pos=np.ascontiguousarray(pos),
        vel=np.ascontiguousarray(vel),
        type=typ,
        ntypes=1,
        pairs=lj_single_pair_table(r_cut),
        seed=seed,
        name=f"lj_fluid_N{n}_rho{rho}",
    )


def make_lj_droplet(
    L: float = 24.0,
    cube: float = 9.0,
    a_dense: float = 0.97,
    a_dilute: float = 1.6,
    T: float = 1.0,
    seed: int = 1,
    jitter: float = 0.05,
) -> LJSystemSpec:
    """Inhomogeneous single-type LJ system: a dense simple-cubic block (spacing ``a_dense``)
    filling the cube [0, cube)^3 of a periodic box of edge ``L``, and a dilute simple-cubic
    vapour (spacing ``a_dilute``, sites at (i + 1/2) a_dilute) everywhere at least a_dilute / 2
    outside that cube, periodically. Cells inside the block hold several times the box's
    mean count, so their bricks' tiles exceed a tile capacity sized for the mean."""
    rng = np.random.default_rng(seed)
    k = int(math.floor(cube / a_dense))
    g = (np.arange(k) + 0.5) * a_dense
    dense = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    m = int(round(L / a_dilute))
    h = (np.arange(m) + 0.5) * (L / m)
    vap = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    gap = 0.5 * a_dilute
    inside = np.all((vap < cube + gap) | (vap >= L - gap), axis=1)
    pos = np.concatenate([dense, vap[~inside]])
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    pos %= L
    n = pos.shape[0]
    vel = _mb_velocities(rng, n, T)
    return LJSystemSpec(
        box=np.array([L, L, L], dtype=np.float64),
        pos=np.ascontiguousarray(pos),
        vel=np.ascontiguousarray(vel),
        type=np.zeros(n, dtype=np.int32),
        ntypes=1,
        pairs=lj_single_pair_table(),
        seed=seed,
        name=f"lj_droplet_L{L}",
    )


def colloid_pair_table(sigma_l: float, cut_factor: float = 2.5):
    """Size-disperse binary LJ mixture: small particles (type 0, sigma 1) and large ones
    (type 1, sigma sigma_l), mixed sigma the arithmetic mean, epsilon 1, r_cut = cut_factor
    sigma_ab (2^(1/6) sigma_ab gives the purely repulsive WCA form)."""
    sig = {(0, 0): 1.0, (0, 1): 0.5 * (1.0 + sigma_l), (1, 1): sigma_l}
    return [(a, b, 1.0, sig[(a, b)], cut_factor * sig[(a, b)]) for (a, b) in sig]


def make_colloid_mixture(
    n_large_side: int = 6,
    sigma_l: float = 3.0,
    spacing_l: float = 5.5,
    rho_small: float = 0.6,
    T: float = 1.0,
    seed: int = 1,
    cut_factor: float = 2.5,
    jitter: float = 0.05,
) -> LJSystemSpec:
    """Size-disperse binary mixture (the case a cell list sized for the largest cutoff serves
    badly): large particles (type 1) on a simple-cubic lattice of n_large_side^3 sites at
    spacing ``spacing_l`` and small particles (type 0) on a simple-cubic lattice at density
    ``rho_small``, without the small sites closer to a large centre than (1 + sigma_l) / 2;
    uniform jitter, Maxwell-Boltzmann velocities at T."""
    rng = np.random.default_rng(seed)
    L = n_large_side * spacing_l
    g = (np.arange(n_large_side) + 0.5) * spacing_l
    large = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    m = int(round(L * rho_small ** (1.0 / 3.0)))
    h = (np.arange(m) + 0.5) * (L / m)
    small = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    excl = 0.5 * (1.0 + sigma_l)
    # the only large centre that can be closer than excl (< spacing_l / 2) is the nearest one
    # of the large lattice: the centre of the lattice cell holding the small site
    if excl >= 0.5 * spacing_l:
        raise ValueError("the large particles' spacing must exceed 1 + sigma_l")
    c = (np.floor(small / spacing_l) + 0.5) * spacing_l
    d = small - c
    keep = (d * d).sum(1) >= excl * excl
    pos = np.concatenate([small[keep], large])
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    pos %= L
    n = pos.shape[0]
    vel = _mb_velocities(rng, n, T)
    typ = np.zeros(n, dtype=np.int32)
    typ[int(keep.sum()):] = 1
    return LJSystemSpec(
        box=np.array([L, L, L], dtype=np.float64),
        pos=np.ascontiguousarray(pos),
        vel=np.ascontiguousarray(vel),
        type=typ,
        ntypes=2,
        pairs=colloid_pair_table(sigma_l, cut_factor),
        seed=seed,
        name=f"colloid_N{n}_sigma{sigma_l}",
    )


def ka_pair_table(cut_factor: float = 2.5):
    """Kob-Andersen 80:20 binary mixture parameters; r_cut = cut_factor * sigma_ab."""
    eps = {(0, 0): 1.0, (0, 1): 1.5, (1, 1): 0.5}
    sig = {(0, 0): 1.0, (0, 1): 0.8, (1, 1): 0.88}
    return [(a, b, eps[(a, b)], sig[(a, b)], cut_factor * sig[(a, b)]) for (a, b) in eps]


def make_ka_mixture(
    n: int, rho: float = 1.2, T: float = 0.45, seed: int = 1, jitter: float = 0.05
) -> LJSystemSpec:
    """Kob-Andersen mixture: N_A = floor(0.8 N + 1/2) type-0 particles, the rest type 1,
    assigned by a seeded permutation drawn after the velocities."""
    rng = np.random.default_rng(seed)
    L = (n / rho) ** (1.0 / 3.0)
    pos = _lattice_positions(rng, n, L, jitter)
    vel = _mb_velocities(rng, n, T)
    n_a = int(math.floor(0.8 * n + 0.5))
    typ = np.ones(n, dtype=np.int32)
    typ[rng.permutation(n)[:n_a]] = 0
    return LJSystemSpec(
        box=np.array([L, L, L], dtype=np.float64),
        pos=np.ascontiguousarray(pos),
        vel=np.ascontiguousarray(vel),
        type=typ,
        ntypes=2,
        pairs=ka_pair_table(),
        seed=seed,
        name=f"ka_N{n}_rho{rho}",
    )


@dataclass
class ReplicaParams:
    n: int
    rho: float
    T: float
    seed: int
    steps: int = 0


def make_replica_specs(count: int = 512, seed: int = 0, n_lo: int = 256, n_hi: int = 8192,
                       rho_lo: float = 0.6, rho_hi: float = 0.9,
                       t_lo: float = 0.8, t_hi: float = 1.5, seed_base: int = 1000):
    """Parameters of independent replicas: N uniform on integers [n_lo, n_hi], density
    uniform on [rho_lo, rho_hi], temperature uniform on [t_lo, t_hi]; replica r uses
    seed ``seed_base + r`` for its own particles."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    rhos = rng.uniform(rho_lo, rho_hi, size=count)
    ts = rng.uniform(t_lo, t_hi, size=count)
    return [ReplicaParams(int(ns[r]), float(rhos[r]), float(ts[r]), seed_base + r)
            for r in range(count)]


def make_arrivals(count: int, rate: float, seed: int = 2, n_lo: int = 512, n_hi: int = 65536,
                  steps_lo: int = 1000, steps_hi: int = 10000, rho: float = 0.8442,
                  T: float = 1.2, seed_base: int = 1_000_000):
    """Poisson request stream: exponential inter-arrival times at ``rate`` per second,
    N log-uniform on [n_lo, n_hi], steps uniform on integers [steps_lo, steps_hi].
    Returns a list of (arrival_time_s, ReplicaParams)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count) if rate > 0 else np.zeros(count)
    times = np.cumsum(gaps)
    logn = rng.uniform(math.log(n_lo), math.log(n_hi), size=count)
    ns = np.clip(np.floor(np.exp(logn)).astype(np.int64), n_lo, n_hi)
    steps = rng.integers(steps_lo, steps_hi + 1, size=count)
    return [(float(times[k]), ReplicaParams(int(ns[k]), rho, T, seed_base + k, int(steps[k])))
            for k in range(count)]
