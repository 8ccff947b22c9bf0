#!/usr/bin/env python3
"""Benchmark of red-black SOR on one MI355X.

Workload (one "step"): a plain FP64 red-black SOR solve of the 4096 x 4096
interior Laplace problem with Dirichlet boundary values drawn uniformly from
[0, 100] (seed 2), omega = 2/(1 + sin(pi/4097)), exactly 1000 iterations with
the stopping rule checked every 10 iterations (tolerance 0, so it never stops
early).  Inputs are resident on the GPU before timing starts; each step runs
through the C ABI (pack into the padded working grids, the blocked sweep
passes with device-side stopping checks, unpack).

Output: one JSON line with GLUP/s (giga lattice-site updates per second), the
dominant kernel's roofline position (algorithmic bytes per launch over the
HIP-event-timed average launch), and the CPU oracle's rate on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blocked_pass_f64_4096.traffic.json")
KERNEL_SOURCES = ("paper_1401_0763_amd/csrc/sor_kernels.h",
                  "paper_1401_0763_amd/csrc/sor_internal.h",
                  "paper_1401_0763_amd/build.py")


def kernel_source_digest():
    """Digest of the sources the blocked sweep kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n, T, seg):
    """Counter-measured bytes per launch, if taken on the current kernel."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("source_digest") != kernel_source_digest():
        return None
    if d.get("config") != {"n": n, "iters_per_pass": T, "seg_rows": seg}:
        return None
    return d["traffic_bytes_per_launch"]
BYTES_PER_LUP_F64 = 16.0       # read u once + write u once per iteration


def cpu_baseline(g, iters_k, seconds):
    """Time the CPU oracle on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    cores = len(os.sched_getaffinity(0))
    threads = max(1, min(cores, 16))
    n = g.n
    calib = 20
    t0 = time.perf_counter()
    oracle.sor_f64(g.u0, g.bdy, None, g.omega, 0.0, calib, iters_k, threads=threads)
    per_iter = (time.perf_counter() - t0) / calib
    iters = int(max(calib, min(20000, seconds / max(per_iter, 1e-9))))
    t0 = time.perf_counter()
    oracle.sor_f64(g.u0, g.bdy, None, g.omega, 0.0, iters, iters_k, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(n * n * iters / dt / 1e9, 4), "unit": "GLUP/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} FP64 Laplace, same seeded inputs, {iters} iterations "
                      f"(check every {iters_k}), OpenMP rows-per-colour workers, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--iters", type=int, default=1000)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one device-to-device copy of this "
                         "many MiB (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the sweep would shard); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1401_0763_amd as sor
    from workloads import laplace_random_boundary

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    n, iters, K = args.n, args.iters, args.check_every
    g = laplace_random_boundary(n, seed=2, max_iters=iters, check_every=K)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    bdy = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
    ctx = sor.context(0)
    T, seg = ctx.get_tiling(64)
    print(f"[bench] n={n} iters={iters} K={K} tiling T={T} seg_rows={seg}",
          file=sys.stderr, flush=True)

    def step():
        return sor.solve_f64(u, bdy, None, g.omega, 0.0, iters, K, ctx=ctx)

    if args.copy_probe_mib:
        nel = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile()
    ctx.set_profiling(False)
    assert res.iterations == iters, res

    glups = n * n * iters * args.steps / dt / 1e9
    avg_launch_s = kern_ms / 1e3 / launches
    alg_bytes = BYTES_PER_LUP_F64 * n * n * T
    achieved = alg_bytes / avg_launch_s / 1e9
    line = {
        "metric": "GLUP/s, 4096^2 FP64 red-black SOR (Laplace, random Dirichlet "
                  "boundary, omega_opt, 1000 iterations checked every 10)",
        "value": round(glups, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded, uniform [0,100] boundary)",
        "config": {"workload": f"laplace_random_boundary_{n}_f64_{iters}it_k{K}",
                   "n": n, "iterations": iters, "check_every": K,
                   "iters_per_pass": T, "seg_rows": seg},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(n, T, seg),
                     "kernel": "blocked_pass_kernel<f64>",
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "launches": launches,
                     "alg_bytes_per_launch": alg_bytes},
        "bandwidth_equiv_GBs": round(glups * BYTES_PER_LUP_F64, 1),
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
