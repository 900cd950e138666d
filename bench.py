#!/usr/bin/env python3
"""Throughput benchmark of the LJ MD hot path on one MI355X.

Workload: single-type LJ fluid, N = 1,048,576, density 0.8442, T = 1.2, r_cut = 2.5
(shifted), skin 0.4, dt = 0.005, velocity-Verlet NVE, synthetic seeded inputs. A "step" is
one full MD step: fused force + integration kernel, gated list rebuild when any particle has
moved skin/2. Timed: exactly --steps steps after --warmup steps, inputs resident in HBM,
bracketed by device synchronisation. Prints ONE JSON line on stdout (progress on stderr).

Also reported on that line:
  roofline      the fused force + integration kernel: algorithmic bytes per launch
                (N * (4 * mean list length + 128)) over its mean launch time, measured with
                HIP events on the library's stream, against 8 TB/s.
  mixed         the same workload with FP32 pair arithmetic (FP64 integration and sums).
  cpu_baseline  the CPU FP64 oracle on a bounded sample of the same workload, on this host.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s: LJ N=1M FP64 vs mixed; batched replicas; serve p50/p99"
HBM_PEAK_GBS = 8000.0
STATE_BYTES = 128  # count 4, x+type 28, v 24, x_build 24 read; x 24, v 24 written


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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
    per_atom = 4.0 * mean_list + STATE_BYTES
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
                     "traffic": None,
                     "kernel": "k_force<fp64, FUSED>", "kernel_avg_ms": fp["kernel_avg_ms"],
                     "bytes_per_atom": fp["bytes_per_atom"]},
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
