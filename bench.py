#!/usr/bin/env python3
"""Throughput benchmark of the LJ MD hot path on one MI355X.

Workload: single-type LJ fluid, N = 1,048,576, density 0.8442, T = 1.2, r_cut = 2.5
(shifted), skin 0.4, dt = 0.005, velocity-Verlet NVE, synthetic seeded inputs. A "step" is
one full MD step: fused force + integration kernel, gated list rebuild when any particle has
moved skin/2. Timed: exactly --steps steps after --warmup steps, inputs resident in HBM,
bracketed by device synchronisation. Prints ONE JSON line on stdout (progress on stderr).

Also reported on that line:
  roofline      the fused force + integration kernel: algorithmic bytes per launch
                (N * (2 * mean list length + 128): 16-bit list entries plus the per-atom
                state) over its mean launch time, measured with HIP events on the library's
                stream, against 8 TB/s.
  mixed         the same workload with FP32 pair arithmetic (FP64 integration and sums).
  batched       512 independent replicas (N uniform in [256, 8192], density in [0.6, 0.9],
                T in [0.8, 1.5]) advanced together in 100-step graph blocks, mixed
                precision, beside a sample of the same replicas run one by one on the plain
                FP64 path.
  served        Poisson request streams (N log-uniform in [512, 65536], density 0.8442,
                T 1.2, 1000-10000 steps) through the continuous-batching loop: p50/p99
                latency and atom-steps/s, beside the same stream served one request at a
                time on the plain FP64 path. Arrival rates are fractions (--serve-loads) of
                the capacity mu = batched atom-steps/s / E[N * steps].
  cpu_baseline  the CPU FP64 oracle on a bounded sample of the same workload, on this host.
"""

import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s: LJ N=1M FP64 vs mixed; batched replicas; serve p50/p99"
HBM_PEAK_GBS = 8000.0
STATE_BYTES = 128  # count 4, x+type 28, v 24, x_build 24 read; x 24, v 24 written
LIST_ENTRY_BYTES = 2  # 16-bit tile index per list entry


def rebuild_bytes(mean_list):
    """Bytes a list rebuild must move per atom: bin (read x 24, write key 4), sort and permute
    (key and index 16, state gather 80 read + 80 written), list write (2 per entry + count 4)."""
    return 28 + 16 + 160 + LIST_ENTRY_BYTES * mean_list + 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_lj_fluid_n1048576_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1308_5587_amd", "csrc", f)
                  for f in ("ljmd_kernels.hip", "ljmd_internal.h")]


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
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line
                  and line.split(": ", 1)[0] in ("launch", "traffic-bytes-per-launch",
                                                 "valu-wave-instructions-per-launch",
                                                 "kernel-source-sha256"))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    if fields.get("kernel-source-sha256", "").strip() != h.hexdigest():
        return None
    if fields.get("launch", "").strip().split(" block=")[0] != f"fp64 tpp={tpp}":
        return None
    return fields


def measured_traffic(tpp, block):
    """HBM bytes per launch of the fused FP64 kernel (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed counter passes, or None (see _counter_fields)."""
    fields = _counter_fields(tpp)
    return float(fields["traffic-bytes-per-launch"]) if fields else None


def valu_issue(tpp, kernel_ms):
    """VALU issue rate of the fused FP64 kernel: the committed count of wave-level VALU
    instructions per launch over the launch time measured here, against the issue peak of one
    VALU instruction per CU per cycle (256 CUs x 2.4 GHz; a wave64 FP64 instruction takes four
    cycles on a 16-lane SIMD, four SIMDs per CU). None without a matching counter pass."""
    fields = _counter_fields(tpp)
    if not fields or "valu-wave-instructions-per-launch" not in fields:
        return None
    insts = float(fields["valu-wave-instructions-per-launch"])
    achieved = insts / (kernel_ms * 1e-3) / 1e9
    peak = 256 * 2.4
    return {"achieved": achieved, "peak": peak, "unit": "G wave-instructions/s",
            "frac": achieved / peak, "instructions_per_launch": insts}


def run_gpu(spec, precision, steps, warmup, timing_steps):
    import torch

    from paper_1308_5587_amd import ljmd

    g = ljmd.System.from_spec(spec, precision=precision)
    g.step(0)  # list, tuning and forces ready
    g.step(warmup)
    st0 = g.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = g.stats()
    wall = t1 - t0
    # dominant kernel: per-launch HIP event timing in a separate pass
    g.set_kernel_timing(True)
    g.step(timing_steps)
    launches, ms = g.kernel_time()
    g.set_kernel_timing(False)
    st2 = g.stats()
    n = spec.n
    mean_list = st2["list_entries"] / n
    per_atom = LIST_ENTRY_BYTES * mean_list + STATE_BYTES
    avg_ms = ms / max(1, launches)
    achieved = n * per_atom / (avg_ms * 1e-3) / 1e9
    rebuilds = st1["rebuilds"] - st0["rebuilds"]
    U, K = g.energy()
    out = {
        "value": n * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "rebuilds": rebuilds,
        "steps_per_rebuild": steps / rebuilds if rebuilds else None,
        "kernel_avg_ms": avg_ms,
        "kernel_launches": launches,
        "mean_list_length": mean_list,
        "bytes_per_atom": per_atom,
        "achieved_gbs": achieved,
        "threads_per_particle": st2["threads_per_particle"],
        "block_size": st2["block_size"],
        "nlist_capacity": st2["nlist_capacity"],
        "energy_per_atom": (U + K) / n,
    }
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


def run_cpu_baseline(spec, steps):
    import oracle

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
                      f"({t1 - t0:.1f} s, excluded), single-threaded FP64 C oracle, "
                      f"{builds} list builds in total"}


def _replica_spec(p, inputs):
    return inputs.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)


def run_alone_timed(spec, nsteps, precision):
    """One replica on the single-system path: wall time of step(nsteps) after setup."""
    import torch

    from paper_1308_5587_amd import ljmd

    g = ljmd.System.from_spec(spec, precision=precision)
    g.step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(nsteps)
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
    b.run_block()  # warm-up block (captures the graph)
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
    # a sample of the same replicas, one by one on the plain FP64 path
    idx = np.random.default_rng(5).choice(count, size=min(sample, count), replace=False)
    work = sum(specs[k].n for k in idx) * block_steps * blocks
    t1 = sum(run_alone_timed(specs[k], block_steps * blocks, "fp64") for k in idx)
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


def run_served(rates, count, block_steps, loads=None):
    from paper_1308_5587_amd import inputs, ljmd, serve

    out = []
    for k, rate in enumerate(rates):
        arrivals = inputs.make_arrivals(count, rate, seed=2)
        mk = lambda p: inputs.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed)  # noqa: E731
        reqs = serve.requests_from_arrivals(arrivals, mk)
        b = ljmd.Batch(16 << 30, 64, precision="mixed", block_steps=block_steps)
        rep = serve.serve(b, reqs).summary()
        b.close()
        log(f"[bench] served rate={rate:.3g}/s: p50 {rep['p50_latency_s']:.3f} s, "
            f"p99 {rep['p99_latency_s']:.3f} s, {rep['atom_steps_per_s']:.4g} atom-steps/s")

        def alone(spec, nsteps):
            g = ljmd.System.from_spec(spec, precision="fp64")
            g.step(nsteps)
            g.close()

        reqs1 = serve.requests_from_arrivals(arrivals, mk)
        base = serve.serve_one_by_one(alone, reqs1).summary()
        log(f"[bench] one by one fp64 rate={rate:.3g}/s: p50 {base['p50_latency_s']:.3f} s, "
            f"p99 {base['p99_latency_s']:.3f} s, {base['atom_steps_per_s']:.4g} atom-steps/s")
        out.append({"rate_per_s": rate, "load": loads[k] if loads else None,
                    "requests": count, **{k: rep[k] for k in (
            "p50_latency_s", "p99_latency_s", "mean_latency_s", "atom_steps_per_s", "wall_s",
            "peak_resident")},
            "one_by_one_fp64": {k: base[k] for k in ("p50_latency_s", "p99_latency_s",
                                                     "atom_steps_per_s", "wall_s")}})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=1_048_576)
    ap.add_argument("--timing-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-blocks", type=int, default=5)
    ap.add_argument("--batched-sample", type=int, default=32)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-drift", action="store_true")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.9",
                    help="arrival rates as fractions of the capacity the batched leg measured")
    ap.add_argument("--serve-rates", type=str, default="",
                    help="explicit arrival rates per second (instead of --serve-loads)")
    ap.add_argument("--serve-count", type=int, default=48)
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
    log(f"[bench] fp64 N={spec.n} steps={args.steps} warmup={args.warmup}")
    fp = run_gpu(spec, "fp64", args.steps, args.warmup, args.timing_steps)
    log(f"[bench] fp64 {fp['value']:.4g} atom-steps/s, {fp['ms_per_step']:.4f} ms/step")
    mixed = None
    if not args.no_mixed:
        log("[bench] mixed")
        mixed = run_gpu(spec, "mixed", args.steps, args.warmup, args.timing_steps)
        log(f"[bench] mixed {mixed['value']:.4g} atom-steps/s")
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
        if args.serve_rates:
            rates = [float(r) for r in args.serve_rates.split(",") if r]
            loads = None
        else:
            # capacity in requests per second: the batched throughput (else the single-system
            # one) over the mean work of a request
            thr = batched["value"] if batched else fp["value"]
            mu = thr / served_mean_work()
            loads = [float(x) for x in args.serve_loads.split(",") if x]
            rates = [x * mu for x in loads]
            log(f"[bench] served: capacity {mu:.3g} requests/s, loads {loads}")
        served = run_served(rates, args.serve_count, 100, loads)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu oracle, {args.cpu_steps} steps")
        cpu = run_cpu_baseline(spec, args.cpu_steps)
        log(f"[bench] cpu {cpu['value']:.4g} atom-steps/s")

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
                   "threads_per_particle": fp["threads_per_particle"],
                   "block_size": fp["block_size"], "steps_per_rebuild": fp["steps_per_rebuild"],
                   "mean_list_length": fp["mean_list_length"]},
        "roofline": {"bound": "hbm", "achieved": fp["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": fp["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(fp["threads_per_particle"], fp["block_size"]),
                     "kernel": "k_force<fp64, FUSED>", "kernel_avg_ms": fp["kernel_avg_ms"],
                     "bytes_per_atom": fp["bytes_per_atom"],
                     "valu_issue": valu_issue(fp["threads_per_particle"], fp["kernel_avg_ms"])},
        "cpu_baseline": cpu,
    }
    if mixed is not None:
        line["mixed"] = {"value": mixed["value"], "ms_per_step": mixed["ms_per_step"],
                         "dtype": "f32 pair / f64 state",
                         "speedup_vs_fp64": mixed["value"] / fp["value"],
                         "roofline_frac": mixed["achieved_gbs"] / HBM_PEAK_GBS,
                         "kernel_avg_ms": mixed["kernel_avg_ms"],
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
    if drift is not None:
        line["energy_drift"] = drift
    if batched is not None:
        line["batched"] = batched
    if served is not None:
        line["served"] = served
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
