"""Short runs of the step loop for profilers (rocprofv3 kernel traces and counter passes).

    python -m paper_1308_5587_amd.profile_run [--n N] [--steps K] [--precision fp64|mixed]
                                              [--tpp T] [--block B] [--copy-mib M]
                                              [--replicas R --blocks K]

First a plain device-to-device copy of M MiB (torch's copy kernel): under a counter pass
its FETCH_SIZE and WRITE_SIZE give the factor between the counters and bytes actually moved.
Then the LJ fluid (density 0.8442, T 1.2, r_cut 2.5, skin 0.4, dt 0.005) is set up with
fixed lanes per particle and workgroup size (so no tuning launches appear in the trace) and
advanced K steps. With --replicas R the batched workload runs instead: R replicas of uneven
size (N uniform in [256, 8192], density in [0.6, 0.9], T in [0.8, 1.5], mixed precision)
admitted into one batch and advanced K blocks of 100 steps. Every step goes through the
library's HIP kernels; one line per phase is printed so a profiler's own output can be
matched to them.
"""

from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--n", type=int, default=1_048_576)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tpp", type=int, default=2)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--replicas", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=2)
    args = ap.parse_args(argv)

    import torch

    from paper_1308_5587_amd import inputs, ljmd

    if not torch.cuda.is_available():
        print("profile_run needs a GPU", file=sys.stderr)
        return 1
    nbytes = args.copy_mib << 20
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[profile] copy {nbytes} bytes read, {nbytes} bytes written", flush=True)
    del src, dst

    if args.replicas:
        params = inputs.make_replica_specs(args.replicas, seed=0)
        specs = [inputs.make_lj_fluid(p.n, rho=p.rho, T=p.T, seed=p.seed) for p in params]
        b = ljmd.Batch(8 << 30, args.replicas, precision="mixed", block_steps=100,
                       threads_per_particle=args.tpp, block_size=args.block)
        for sp in specs:
            b.admit(sp, 100 * args.blocks)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.blocks):
            b.run_block()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = b.stats()
        print(f"[profile] batched replicas={args.replicas} atoms={sum(s.n for s in specs)} "
              f"blocks={args.blocks} tpp={st['threads_per_particle']} "
              f"block={st['block_size']} wall={dt:.4f}s rebuilds={st['rebuilds']}", flush=True)
        b.close()
        return 0

    spec = inputs.make_lj_fluid(args.n, rho=0.8442, T=1.2, seed=1)
    g = ljmd.System.from_spec(spec, precision=args.precision, threads_per_particle=args.tpp,
                              block_size=args.block)
    g.step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = g.stats()
    print(f"[profile] {args.precision} n={spec.n} steps={args.steps} tpp={args.tpp} "
          f"block={args.block} wall={dt:.4f}s rebuilds={st['rebuilds']} "
          f"mean_list={st['list_entries'] / spec.n:.2f}", flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
