#!/usr/bin/env python3
"""Throughput benchmark of the LJ MD hot path on one MI355X.

Headline workload: single-type LJ fluid, N = 1,048,576, density 0.8442, T = 1.2, r_cut = 2.5
(shifted), skin 0.4, dt = 0.005, velocity-Verlet NVE, FP64, synthetic seeded inputs. A "step"
is one full MD step: the fused force + integration kernel and the list-rebuild kernels,
which rebuild when any particle has moved skin/2. Timed: exactly --steps steps after
--warmup steps, inputs resident in HBM, bracketed by device synchronisation, with the
energy, kinetic energy and virial reduced every --thermo-period steps inside the timed
loop. Prints ONE JSON line on stdout (progress on stderr).

Also reported on that line:
  kernels       per-step time of each kernel class, from HIP events around every launch in
                a separate pass: the step kernel, the list build and the other rebuild
                kernels when they rebuild (amortised over the steps), and the same kernels
                when they return at once (no rebuild asked).
  roofline      the dominant kernel (largest per-step time): algorithmic bytes per launch
                over its mean launch time against 8 TB/s; `roofline_kernels` holds the
                figure for both the fused step kernel and the list build.
  mixed         the same workload with FP32 pair arithmetic (FP64 integration and sums).
  lj_fluid_N4000   the small correctness workload (N = 4000, FP64, 100 steps): time per step.
  ka_mixture    the Kob-Andersen mixture (N = 262,144, density 1.2, per-pair cutoffs),
                mixed precision, 2000 steps: atom-steps/s and its fused kernel's roofline.
  paper_benchmark  the paper's LJ liquid benchmark (N = 64,000, density 0.382,
                r_cut = 3.0, NVT kT = 1.2, tau = 1.0, dt = 0.005), beside the paper's own
                figures for other hardware (context only).
  size_disperse a size-disperse LJ mixture (size ratio 3:1, N = 1.1 M, of which 13,824 large),
                FP64, with the cell list and with the tree lists: atom-steps/s of each and
                the list build's per-build time.
  batched       512 independent replicas (N uniform in [256, 8192], density in [0.6, 0.9],
                T in [0.8, 1.5]) advanced together in 100-step graph blocks, mixed
                precision, beside a sample of the same replicas run one by one on the plain
                FP64 path.
  served        Poisson request streams (N log-uniform in [512, 65536], density 0.8442,
                T 1.2, 1000-10000 steps) through the continuous-batching loop under a memory
                budget that limits admission: p50/p99 latency and atom-steps/s at arrival
                rates that are fractions of the capacity mu = batched atom-steps/s /
                E[N * steps]; beside the same stream served one request at a time on the
                plain FP64 path (each request's measured alone time replayed through the
                same first-come first-served queue).
  cpu_baseline  the CPU FP64 oracle on a bounded sample of the headline workload, on this
                host (core count and CPU model stated).
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s: LJ N=1M FP64 vs mixed; batched replicas; serve p50/p99"
HBM_PEAK_GBS = 8000.0
# fused step kernel, per atom: list count 4, x+type 28, v 24, x_build 24 read; x 24, v 24
# written; plus 2 bytes per 16-bit list entry
STATE_BYTES = 128
LIST_ENTRY_BYTES = 2
# list build, per atom: the permuted state read (x 32, v 32, images and tag 16) and written
# back with the build positions (x 32, x_build 32, v 32, images 16), the count 4 and the
# work-order entry 2; plus 2 bytes per list entry written
NLIST_STATE_BYTES = 80 + 112 + 4 + 2
# list build, per candidate pair the cell method tests (every atom of the 27 stencil cells of
# the particle's cell): the canonical FP64 distance test, 3 differences, 3 products, 2 sums
# and one comparison. Peak for such single FP64 operations: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3 T operations/s (the published 78.6 TFLOP/s counts a multiply-add as two).
NLIST_OPS_PER_TEST = 9
FP64_OPS_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
PAPER_CONTEXT = {"xeon_platinum_8160_24_cores": 16.1e6, "v100_fp64": 2.75e8,
                 "unit": "particle-steps/s", "source": "paper, Section Performance"}


def rebuild_bytes(mean_list):
    """Bytes a list rebuild must move per atom: bin (read x 24, write key 4), sort and permute
    (key and index 16, state gather 80 read + 80 written), list write (2 per entry + count 4)."""
    return 28 + 16 + 160 + LIST_ENTRY_BYTES * mean_list + 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_lj_fluid_n1048576_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1308_5587_amd", "csrc", f)
                  for f in ("ljmd_kernels.hip", "ljmd_internal.h", "ljmd_device.h", "ljmd_force.h",
                            "ljmd_force_lj.hip")]


def _counter_fields(tpp):
    """Machine-readable lines of the committed counter passes over the fused FP64 kernel, if
    they were taken on the current kernel sources with these lanes per particle; else None.
    The workgroup size is not matched: one workgroup per brick moves the same bytes and issues
    the same instructions at any size."""
    import hashlib

    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    keys = ("launch", "traffic-bytes-per-launch", "valu-wave-instructions-per-launch",
            "kernel-source-sha256", "nlist-traffic-bytes-per-build",
            "nlist-valu-wave-instructions-per-build")
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line
                  and line.split(": ", 1)[0] in keys)
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    if fields.get("kernel-source-sha256", "").strip() != h.hexdigest():
        return None
    if fields.get("launch", "").strip().split(" block=")[0] != f"fp64 tpp={tpp}":
        return None
    return fields


def valu_issue(insts, kernel_ms):
    """VALU issue rate: wave-level VALU instructions per launch over the launch time measured
    here, against the issue peak of one VALU instruction per CU per cycle (256 CUs x 2.4 GHz;
    a wave64 FP64 instruction takes four cycles on a 16-lane SIMD, four SIMDs per CU)."""
    achieved = insts / (kernel_ms * 1e-3) / 1e9
    peak = 256 * 2.4
    return {"achieved": achieved, "peak": peak, "unit": "G wave-instructions/s",
            "frac": achieved / peak, "instructions_per_launch": insts}


def kernel_breakdown(durations, units):
    """Per-step milliseconds of each kernel class from per-launch durations of `units` timed
    steps. A unit rebuilt the list when its list-build launch was far longer than the median
    (most steps do not rebuild, and their gated launches return at once)."""
    nl = durations["nlist"]
    thr = 5.0 * float(np.median(nl))
    active = nl > thr
    out = {"units": int(units), "rebuilds": int(active.sum()),
           "step_kernel": float(durations["step"].sum() / units),
           "step_kernel_avg": float(durations["step"].mean())}
    other = ("bin", "scan", "scatter", "gather")
    out["build_active"] = float(nl[active].sum() / units)
    out["other_rebuild_active"] = float(sum(durations[k][active].sum() for k in other) / units)
    out["gated_idle"] = float(sum(durations[k][~active].sum() for k in other + ("nlist",)) / units)
    out["per_build"] = {k: float(durations[k][active].mean()) if active.any() else None
                        for k in other + ("nlist",)}
    out["per_idle_launch"] = {k: float(durations[k][~active].mean()) if (~active).any() else None
                              for k in other + ("nlist",)}
    out["unit"] = "ms per step (per launch for per_build / per_idle_launch)"
    return out


def run_gpu(spec, precision, steps, warmup, timing_steps, thermo_period=0, nvt=None,
            nlist="cell"):
    """Time `steps` steps of one system; then a separate pass with events around every kernel
    launch. thermo_period > 0 reduces U, K and W every that many steps inside the timed loop."""
    import torch

    from paper_1308_5587_amd import ljmd

    g = ljmd.System.from_spec(spec, precision=precision)
    if nlist != "cell":
        g.set_nlist(nlist)
    if nvt:
        g.set_nvt(*nvt)
    g.step(0)  # list, tuning and forces ready
    g.step(warmup)
    st0 = g.stats()
    chunk = thermo_period if thermo_period > 0 else steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        g.step(k)
        done += k
        if thermo_period > 0:
            g.energy()
            g.virial()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = g.stats()
    wall = t1 - t0
    out = {"value": spec.n * steps / wall, "ms_per_step": 1e3 * wall / steps,
           "rebuilds": st1["rebuilds"] - st0["rebuilds"]}
    out["steps_per_rebuild"] = steps / out["rebuilds"] if out["rebuilds"] else None
    if timing_steps > 0:
        g.set_kernel_timing(True)
        g.step(timing_steps)
        d = g.kernel_durations()
        g.set_kernel_timing(False)
        units = len(d["step"])
        out["kernels"] = kernel_breakdown(d, units)
    st2 = g.stats()
    n = spec.n
    mean_list = st2["list_entries"] / n
    out.update({"mean_list_length": mean_list,
                "threads_per_particle": st2["threads_per_particle"],
                "block_size": st2["block_size"], "nlist_capacity": st2["nlist_capacity"]})
    if timing_steps > 0:
        kb = out["kernels"]
        per_atom = LIST_ENTRY_BYTES * mean_list + STATE_BYTES
        out["step_kernel_bytes_per_atom"] = per_atom
        out["step_kernel_gbs"] = n * per_atom / (kb["step_kernel_avg"] * 1e-3) / 1e9
        nb = kb["per_build"]["nlist"]
        out["nlist_bytes_per_atom"] = LIST_ENTRY_BYTES * mean_list + NLIST_STATE_BYTES
        out["nlist_gbs"] = (n * out["nlist_bytes_per_atom"] / (nb * 1e-3) / 1e9) if nb else None
        ncell = int(np.prod(st2["ncell"]))
        out["nlist_tests_per_atom"] = 27.0 * n / ncell
        out["nlist_tops"] = (n * out["nlist_tests_per_atom"] * NLIST_OPS_PER_TEST / (nb * 1e-3)
                             / 1e12) if nb else None
    U, K = g.energy()
    out["energy_per_atom"] = (U + K) / n
    g.close()
    return out


def energy_drift(spec, precision, steps, every, dt=0.005):
    """NVE energy drift: least-squares slope of (E(t) - E(0)) / N against t / tau over
    `steps` steps sampled every `every` steps, and the RMS of (E - E(0)) / N."""
    from paper_1308_5587_amd import ljmd

    g = ljmd.System.from_spec(spec, precision=precision)
    U, K = g.energy()
    e0 = U + K
    t, de = [0.0], [0.0]
    for k in range(every, steps + 1, every):
        g.step(every)
        U, K = g.energy()
        t.append(k * dt)
        de.append((U + K - e0) / spec.n)
    st = g.stats()
    g.close()
    t = np.array(t)
    de = np.array(de)
    slope = float(np.polyfit(t, de, 1)[0])
    return {"drift_per_atom_per_tau": slope, "rms_per_atom": float(np.sqrt(np.mean(de ** 2))),
            "tau": steps * dt, "steps": steps, "samples": len(t), "rebuilds": st["rebuilds"],
            "e0_per_atom": e0 / spec.n}


def _host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "model": model}


def run_cpu_baseline(spec, steps):
    import oracle

    oracle.use_native_build()
    t0 = time.perf_counter()
    o = oracle.OracleSystem.from_spec(spec)
    o.compute()
    t1 = time.perf_counter()
    o.step(steps)
    t2 = time.perf_counter()
    _, builds = o.counters()
    return {"value": spec.n * steps / (t2 - t1), "unit": "atom-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"N={spec.n} fluid, {steps} NVE steps after the initial list build "
                      f"({t1 - t0:.1f} s, excluded), {t2 - t1:.1f} s, single-threaded FP64 C "
                      f"oracle, {builds} list builds in total",
            "build": oracle.build_flags(native=True), "host": _host_cpu()}


def _replica_spec(p, inputs):
    return inputs.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)


def run_alone_timed(spec, nsteps, precision):
    """One replica on the single-system path: wall time of create + step(nsteps) + reading
    its results, as a request served alone takes it."""
    import torch

    from paper_1308_5587_amd import ljmd

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ljmd.System.from_spec(spec, precision=precision)
    g.step(nsteps)
    g.state()
    g.forces()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    return dt


def run_batched(count, block_steps, blocks, sample):
    import torch

    from paper_1308_5587_amd import inputs, ljmd

    params = inputs.make_replica_specs(count, seed=0)
    specs = [_replica_spec(p, inputs) for p in params]
    atoms = sum(s.n for s in specs)
    nsteps = (blocks + 1) * block_steps
    probe = ljmd.Batch(1 << 30, 1, precision="mixed", block_steps=block_steps)
    budget = int(1.25 * sum(probe.footprint(s) for s in specs)) + (64 << 20)
    probe.close()
    b = ljmd.Batch(budget, count, precision="mixed", block_steps=block_steps)
    t0 = time.perf_counter()
    slots = [b.admit(s, nsteps) for s in specs]
    torch.cuda.synchronize()
    t_admit = time.perf_counter() - t0
    b.run_block()  # warm-up block (tunes, captures the graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(blocks):
        b.run_block()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert len(b.poll()) == count
    for s in slots:
        assert b.slot_steps(s) == nsteps
    bst = b.stats()
    b.close()
    # a sample of the same replicas, one by one on the plain FP64 path (steps only)
    idx = np.random.default_rng(5).choice(count, size=min(sample, count), replace=False)
    work = sum(specs[k].n for k in idx) * block_steps * blocks
    t1 = 0.0
    for k in idx:
        g = ljmd.System.from_spec(specs[k], precision="fp64")
        g.step(0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        g.step(block_steps * blocks)
        torch.cuda.synchronize()
        t1 += time.perf_counter() - ts
        g.close()
    value = atoms * block_steps * blocks / wall
    alone = work / t1
    return {"value": value, "unit": "atom-steps/s", "replicas": count, "atoms": atoms,
            "block_steps": block_steps, "blocks": blocks, "ms_per_block": 1e3 * wall / blocks,
            "admit_s": t_admit, "dtype": "f32 pair / f64 state",
            "threads_per_particle": bst["threads_per_particle"], "block_size": bst["block_size"],
            "tile_capacity": bst["tile_capacity"], "rebuilds": bst["rebuilds"],
            "one_by_one_fp64": {"value": alone, "unit": "atom-steps/s", "replicas": len(idx),
                                "steps": block_steps * blocks},
            "speedup_vs_one_by_one_fp64": value / alone}


def served_mean_work():
    """E[N x steps] of the request stream (N log-uniform on [512, 65536], steps uniform on
    [1000, 10000], drawn independently)."""
    n_lo, n_hi, s_lo, s_hi = 512, 65536, 1000, 10000
    return (n_hi - n_lo) / math.log(n_hi / n_lo) * 0.5 * (s_lo + s_hi)


def fifo_replay(arrivals, service):
    """Latencies of requests served one at a time, first come first served, each taking its
    measured service time."""
    free = 0.0
    lat = []
    for t, s in zip(arrivals, service):
        start = max(t, free)
        free = start + s
        lat.append(free - t)
    return np.array(lat), free


def run_served(loads, mu, count, block_steps, budget, max_slots):
    from paper_1308_5587_amd import inputs, ljmd, serve

    mk = lambda p: inputs.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)  # noqa: E731
    out = []
    work = None
    for load in loads:
        rate = load * mu
        arrivals = inputs.make_arrivals(count, rate, seed=2)
        reqs = serve.requests_from_arrivals(arrivals, mk)
        work = [(r.n, r.nsteps) for r in reqs]
        b = ljmd.Batch(budget, max_slots, precision="mixed", block_steps=block_steps)
        rep = serve.serve(b, reqs)
        b.close()
        s = rep.summary()
        log(f"[bench] served load {load} ({rate:.3g}/s): p50 {s['p50_latency_s']:.3f} s, "
            f"p99 {s['p99_latency_s']:.3f} s, {s['atom_steps_per_s']:.4g} atom-steps/s, "
            f"peak resident {s['peak_resident']}, {s['refused_for_capacity']} refused for "
            f"capacity at least once")
        out.append({"load": load, "rate_per_s": rate, "requests": count,
                    **{k: s[k] for k in ("p50_latency_s", "p99_latency_s", "mean_latency_s",
                                         "atom_steps_per_s", "wall_s", "peak_resident",
                                         "failed", "refused_for_capacity")},
                    "_arrivals": [t for t, _ in arrivals]})
    # one by one on the plain FP64 path: every request's alone time, measured once (the
    # request sizes and step counts do not depend on the rate), replayed through the queue
    log(f"[bench] served: measuring {count} requests alone on the FP64 path")
    arrivals = inputs.make_arrivals(count, 1.0, seed=2)
    service = [run_alone_timed(mk(p), p.steps, "fp64") for _, p in arrivals]
    for o in out:
        lat, end = fifo_replay(o.pop("_arrivals"), service)
        o["one_by_one_fp64"] = {
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "atom_steps_per_s": float(sum(n * k for n, k in work) / end),
            "method": "measured alone service times replayed first come first served"}
    return {"budget_bytes": budget, "max_slots": max_slots, "capacity_requests_per_s": mu,
            "mean_request_work_atom_steps": served_mean_work(), "loads": out,
            "alone_service_s": {"mean": float(np.mean(service)), "sum": float(np.sum(service))}}


def _roof(name, gbs, avg_ms, bytes_per_atom, n, per_step_ms, valu=None, traffic=None):
    r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": name,
         "kernel_avg_ms": avg_ms, "bytes_per_atom": bytes_per_atom, "atoms_per_launch": n,
         "ms_per_step": per_step_ms}
    if valu is not None:
        r["valu_issue"] = valu
    return r


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=1_048_576)
    ap.add_argument("--thermo-period", type=int, default=100)
    ap.add_argument("--timing-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the N=4000, KA and paper legs")
    ap.add_argument("--size-disperse-steps", type=int, default=200)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-blocks", type=int, default=10)
    ap.add_argument("--batched-sample", type=int, default=32)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-drift", action="store_true")
    ap.add_argument("--serve-loads", type=str, default="0.25,0.5,0.75,0.9,1.0,1.2",
                    help="arrival rates as fractions of the capacity the batched leg measured")
    ap.add_argument("--serve-count", type=int, default=100)
    ap.add_argument("--serve-budget-mib", type=int, default=384)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: multi-GPU runs (--gpus > 1) are not part of "
              "this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1308_5587_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    spec = inputs.make_lj_fluid(args.n, rho=0.8442, T=1.2, seed=1)
    log(f"[bench] fp64 N={spec.n} steps={args.steps} warmup={args.warmup} "
        f"thermo every {args.thermo_period}")
    fp = run_gpu(spec, "fp64", args.steps, args.warmup, args.timing_steps, args.thermo_period)
    kb = fp["kernels"]
    log(f"[bench] fp64 {fp['value']:.4g} atom-steps/s, {fp['ms_per_step']:.4f} ms/step; "
        f"step kernel {kb['step_kernel']:.4f}, build {kb['build_active']:.4f}, other rebuild "
        f"{kb['other_rebuild_active']:.4f}, idle gated {kb['gated_idle']:.4f} ms/step")
    mixed = None
    if not args.no_mixed:
        log("[bench] mixed")
        mixed = run_gpu(spec, "mixed", args.steps, args.warmup, args.timing_steps,
                        args.thermo_period)
        log(f"[bench] mixed {mixed['value']:.4g} atom-steps/s")
    configs = {}
    if not args.no_configs:
        small = inputs.make_lj_fluid(4000, rho=0.8442, T=1.2, seed=1)
        c1 = run_gpu(small, "fp64", 100, 20, 0)
        configs["lj_fluid_N4000"] = {"ms_per_step": c1["ms_per_step"], "value": c1["value"],
                                     "steps": 100, "dtype": "f64", "note": "cache-resident"}
        log(f"[bench] N=4000 fp64: {c1['ms_per_step']:.4f} ms/step")
        ka = inputs.make_ka_mixture(262_144, seed=1)
        c3 = run_gpu(ka, "mixed", 2000, 50, args.timing_steps)
        configs["ka_mixture_N262144"] = {
            "value": c3["value"], "ms_per_step": c3["ms_per_step"], "steps": 2000,
            "dtype": "f32 pair / f64 state", "steps_per_rebuild": c3["steps_per_rebuild"],
            "mean_list_length": c3["mean_list_length"], "kernels": c3["kernels"],
            "roofline": _roof("k_force<mixed, FUSED, multi-type>", c3["step_kernel_gbs"],
                              c3["kernels"]["step_kernel_avg"], c3["step_kernel_bytes_per_atom"],
                              ka.n, c3["kernels"]["step_kernel"])}
        log(f"[bench] KA N=262144 mixed: {c3['value']:.4g} atom-steps/s")
        pb = inputs.make_lj_fluid(64000, rho=0.382, T=1.2, seed=1, r_cut=3.0)
        c6 = run_gpu(pb, "fp64", 2000, 100, args.timing_steps, nvt=(1.2, 1.0))
        configs["paper_lj_liquid_N64000_nvt"] = {
            "value": c6["value"], "ms_per_step": c6["ms_per_step"], "steps": 2000,
            "dtype": "f64", "ensemble": "nvt kT=1.2 tau=1.0", "density": 0.382, "r_cut": 3.0,
            "steps_per_rebuild": c6["steps_per_rebuild"], "kernels": c6["kernels"],
            "paper_context": PAPER_CONTEXT}
        log(f"[bench] paper benchmark N=64000 NVT fp64: {c6['value']:.4g} atom-steps/s")
        cm = inputs.make_colloid_mixture(n_large_side=24, sigma_l=3.0)
        sd = {}
        for method in ("tree", "cell"):
            r = run_gpu(cm, "fp64", args.size_disperse_steps, 20, 100, nlist=method)
            sd[method] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                          "steps_per_rebuild": r["steps_per_rebuild"],
                          "mean_list_length": r["mean_list_length"],
                          "build_ms": r["kernels"]["per_build"]["nlist"],
                          "step_kernel_ms": r["kernels"]["step_kernel_avg"],
                          "threads_per_particle": r["threads_per_particle"]}
            log(f"[bench] size-disperse N={cm.n} {method}: {r['value']:.4g} atom-steps/s, "
                f"build {sd[method]['build_ms']} ms")
        configs["size_disperse_N%d" % cm.n] = {
            "n": cm.n, "n_large": int((cm.type == 1).sum()), "size_ratio": 3.0,
            "steps": args.size_disperse_steps, "dtype": "f64", **sd,
            "tree_speedup_vs_cell": sd["tree"]["value"] / sd["cell"]["value"]}
    drift = None
    if not args.no_drift:
        log("[bench] energy drift: N=2^20 over 5 tau, N=4000 over 100 tau")
        small = inputs.make_lj_fluid(4000, rho=0.8442, T=1.2, seed=1)
        drift = {"lj_fluid_N1048576": {p: energy_drift(spec, p, 1000, 50)
                                       for p in ("fp64", "mixed")},
                 "lj_fluid_N4000": {p: energy_drift(small, p, 20000, 200)
                                    for p in ("fp64", "mixed")}}
        for w, d in drift.items():
            for p, v in d.items():
                log(f"[bench] drift {w} {p}: {v['drift_per_atom_per_tau']:.3e} per atom per tau, "
                    f"rms {v['rms_per_atom']:.3e}")
    batched = None
    if not args.no_batched:
        log("[bench] batched: 512 replicas")
        batched = run_batched(512, 100, args.batched_blocks, args.batched_sample)
        log(f"[bench] batched {batched['value']:.4g} atom-steps/s "
            f"(one by one fp64 {batched['one_by_one_fp64']['value']:.4g})")
    served = None
    if not args.no_serve:
        thr = batched["value"] if batched else fp["value"]
        mu = thr / served_mean_work()
        loads = [float(x) for x in args.serve_loads.split(",") if x]
        log(f"[bench] served: capacity {mu:.3g} requests/s, loads {loads}")
        served = run_served(loads, mu, args.serve_count, 100, args.serve_budget_mib << 20, 64)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu oracle, {args.cpu_steps} steps")
        cpu = run_cpu_baseline(spec, args.cpu_steps)
        log(f"[bench] cpu {cpu['value']:.4g} atom-steps/s")

    fields = _counter_fields(fp["threads_per_particle"])
    step_valu = (valu_issue(float(fields["valu-wave-instructions-per-launch"]),
                            kb["step_kernel_avg"])
                 if fields and "valu-wave-instructions-per-launch" in fields else None)
    nl_avg = kb["per_build"]["nlist"]
    nl_valu = (valu_issue(float(fields["nlist-valu-wave-instructions-per-build"]), nl_avg)
               if fields and "nlist-valu-wave-instructions-per-build" in fields and nl_avg
               else None)
    roof_step = _roof("k_force<fp64, FUSED>", fp["step_kernel_gbs"], kb["step_kernel_avg"],
                      fp["step_kernel_bytes_per_atom"], spec.n, kb["step_kernel"], step_valu,
                      float(fields["traffic-bytes-per-launch"]) if fields else None)
    roof_nl = None
    if nl_avg:
        # the build is bound by its FP64 distance tests (ALU), not by its bytes: reported
        # against the FP64 operation peak, with its HBM view beside it
        roof_nl = {"bound": "alu", "achieved": fp["nlist_tops"], "peak": FP64_OPS_PEAK_T,
                   "unit": "TFLOP/s", "frac": fp["nlist_tops"] / FP64_OPS_PEAK_T,
                   "traffic": (float(fields["nlist-traffic-bytes-per-build"])
                               if fields and "nlist-traffic-bytes-per-build" in fields
                               else None),
                   "kernel": "k_nlist (list build)", "kernel_avg_ms": nl_avg,
                   "tests_per_atom": fp["nlist_tests_per_atom"],
                   "ops_per_test": NLIST_OPS_PER_TEST, "atoms_per_launch": spec.n,
                   "ms_per_step": kb["build_active"],
                   "hbm": {"achieved": fp["nlist_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": fp["nlist_gbs"] / HBM_PEAK_GBS,
                           "bytes_per_atom": fp["nlist_bytes_per_atom"]}}
        if nl_valu is not None:
            roof_nl["valu_issue"] = nl_valu
    dominant = roof_nl if (roof_nl and kb["build_active"] > kb["step_kernel"]) else roof_step
    line = {
        "metric": METRIC,
        "value": fp["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lj_fluid_N1048576_rho0.8442_fp64_nve", "n": spec.n,
                   "density": 0.8442, "T0": 1.2, "r_cut": 2.5, "skin": 0.4, "dt": 0.005,
                   "thermo_period": args.thermo_period,
                   "threads_per_particle": fp["threads_per_particle"],
                   "block_size": fp["block_size"], "steps_per_rebuild": fp["steps_per_rebuild"],
                   "mean_list_length": fp["mean_list_length"]},
        "roofline": dominant,
        "roofline_kernels": [r for r in (roof_step, roof_nl) if r],
        "kernels": kb,
        "cpu_baseline": cpu,
    }
    if mixed is not None:
        line["mixed"] = {"value": mixed["value"], "ms_per_step": mixed["ms_per_step"],
                         "dtype": "f32 pair / f64 state",
                         "speedup_vs_fp64": mixed["value"] / fp["value"],
                         "roofline_frac": mixed["step_kernel_gbs"] / HBM_PEAK_GBS,
                         "kernels": mixed["kernels"],
                         "threads_per_particle": mixed["threads_per_particle"],
                         "block_size": mixed["block_size"]}
    # the whole step against the method's bytes: list + state every step, rebuild amortised
    k_bar = fp["steps_per_rebuild"] or float("inf")
    b_step = (LIST_ENTRY_BYTES * fp["mean_list_length"] + 4 + (STATE_BYTES - 4)
              + rebuild_bytes(fp["mean_list_length"]) / k_bar)
    line["path_roofline"] = {"bound": "hbm", "bytes_per_atom_step": b_step,
                             "ceiling_atom_steps_per_s": HBM_PEAK_GBS * 1e9 / b_step,
                             "frac": fp["value"] / (HBM_PEAK_GBS * 1e9 / b_step),
                             "mixed_frac": (mixed["value"] / (HBM_PEAK_GBS * 1e9 / b_step)
                                            if mixed else None)}
    if configs:
        line["configs"] = configs
    if drift is not None:
        line["energy_drift"] = drift
    if batched is not None:
        line["batched"] = batched
    if served is not None:
        line["served"] = served
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
