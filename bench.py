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
dominant kernel's roofline position, and the CPU oracle's rate on the host
cores.  The sweep applies 7 iterations per pass over HBM, so HBM traffic is
a fraction of the algorithmic bytes: the roofline reports the update's FP64
floating-point operations (9 per lattice update, a fused multiply-add
counting two: three adds for the neighbour sum, the quarter-difference and
the relaxation step as two fused multiply-adds, the change and its running
maximum) over the HIP-event-timed kernel time, against the chip's FP64
vector peak of 78.6 TFLOP/s (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4
GHz).  Beside it: the same work in issue slots (7 FP64 vector instructions
per update against 39.3 T instructions/s), the HBM-equivalent bandwidth (16
algorithmic bytes per update), the counter-measured HBM traffic per launch
with its bandwidth and fraction of the 8 TB/s peak, and the achievable
bandwidth of a 1 GiB device copy.  Every timed step starts from the zero
interior of the workload.  The CPU baseline is the oracle on up to 16 host
threads, with its single-thread rate and the CPU model beside it.
Under "forms" the same line reports:
  tol      the benchmark grid solved to max |du| < 1e-8 (checked every 10);
  paper    the paper's own configuration (omega 0.376, north edge 1, other
           edges 0, tol 1e-5 checked every 4000 iterations, at most 50000),
           with the iteration count the paper does not print;
  control_8192  8192^2, 300 iterations: grids beyond the Infinity Cache;
  3d       the 3-D extension (7-point stencil), 256^3, 1000 iterations and
           to 1e-8, with the CPU oracle timed on 200 iterations;
  variants the Jacobi and four-colour orderings and block-parallel SOR
           (128 x 128 blocks) on 4096^2 (200 iterations) and iterations to
           1e-8 on 128^2 beside red-black;
and, each against plain one-grid-at-a-time FP64 on the same GPU:
  mixed    4096^2 Poisson (f = N(0,1) + 2 pi^2 sin sin, seed 3): FP64 defect
           correction around FP32 inner sweeps vs plain FP64 SOR, each run to
           its accuracy floor: relative residual, normwise backward error,
           error against the exact discrete solution (DST-I) and difference
           from the FP64 SOR result, update rates (GLUP/s) and algorithmic
           bandwidth; binary16 inner storage at 1024^2 (the largest side it
           accepts) beside FP32 there;
  batched  512 grids, sides log-uniform in [64, 1024] (seed 4), f = N(0,1) on
           odd grids, omega_opt, tol 1e-8: one persistent launch, FP64 (with
           the size rule's tiles and with autotuned tiles) and
           FP32+refinement, solves/s;
  serving  Poisson arrivals (seed 5) of requests with sides log-uniform in
           [128, 2048], boundary U[0,100], f = N(0,1), each to relative
           residual 1e-8 by FP32 + FP64 refinement through the request server,
           at 0.7 x the server's saturated rate: p50/p99 latency and solves/s.
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
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector peak (fused multiply-add = 2 flops)
FP64_VALU_ISSUE_TIPS = 256 * 4 * 16 * 2.4e9 / 1e12   # FP64 vector instructions/s, 39.3 T
FLOPS_PER_LUP_F64 = 9          # 3 adds + 2 fused multiply-adds (2 each) + change + max
INSTR_PER_LUP_F64 = 7          # the same as FP64 vector instructions
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


def copy_bandwidth(torch, mib=1024, reps=5):
    """Achievable HBM bandwidth: a device elementwise copy of `mib` MiB of
    FP64 (read + write), median of `reps` event-timed runs."""
    src = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.add(src, 0.0, out=dst)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.add(src, 0.0, out=dst)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    t = sorted(times)[len(times) // 2]
    return round(2 * mib * (1 << 20) / t / 1e9, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    iters1 = max(2, iters // (4 * threads))      # about a quarter as long at linear scaling
    t0 = time.perf_counter()
    oracle.sor_f64(g.u0, g.bdy, None, g.omega, 0.0, iters1, iters_k, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(n * n * iters / dt / 1e9, 4), "unit": "GLUP/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} FP64 Laplace, same seeded inputs, {iters} iterations "
                      f"(check every {iters_k}), OpenMP rows-per-colour workers, "
                      f"{dt:.1f} s",
            "value_1_thread": round(n * n * iters1 / dt1 / 1e9, 4),
            "sample_1_thread": f"same grid, {iters1} iterations, {dt1:.1f} s",
            "cpu_model": cpu_model()}


def dst_exact(n, bdy, f):
    """Exact discrete solution of the 5-point Dirichlet problem (DST-I)."""
    import numpy as np
    import scipy.fft
    h = 1.0 / (n + 1)
    b = rhs_b(n, bdy, f)
    s2 = np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    lam = 4.0 * (s2[:, None] + s2[None, :])
    return scipy.fft.idstn(scipy.fft.dstn(b, type=1, norm="ortho") / lam, type=1,
                           norm="ortho")


def fp64_to_residual(sor, ctx, u, b, f, omega, rel_tol, chunk, max_iters, trace=None):
    """Plain FP64 SOR from u, checking the relative residual every `chunk`
    iterations; returns (iterations, rel).  trace, if a list, receives
    (seconds, iterations, rel) after every chunk."""
    its, rel = 0, float("inf")
    t0 = time.perf_counter()
    while its < max_iters:
        sor.solve_f64(u, b, f, omega, 0.0, chunk, chunk, ctx=ctx)
        its += chunk
        sr, sb, _ = sor.residual_f64(u, b, f, ctx=ctx)
        rel = math.sqrt(sr) / math.sqrt(sb) if sb > 0 else math.sqrt(sr)
        if trace is not None:
            trace.append((time.perf_counter() - t0, its, rel))
        if rel <= rel_tol:
            break
    return its, rel


def time_to(trace, target):
    """First time in a (seconds, work, rel) trace at which rel <= target."""
    for t, _, r in trace:
        if r <= target:
            return round(t, 3)
    return None


def rhs_b(n, bdy, f):
    """b = h*h*f + (boundary neighbours) of the h*h-scaled 5-point system."""
    import numpy as np
    h = 1.0 / (n + 1)
    b = h * h * np.asarray(f, dtype=np.float64).copy()
    b[0, :] += bdy[0:n]
    b[-1, :] += bdy[n:2 * n]
    b[:, 0] += bdy[2 * n:3 * n]
    b[:, -1] += bdy[3 * n:4 * n]
    return b


def accuracy(sor, ctx, u, b_dev, f_dev, b_inf, exact, scale, ref=None):
    """Relative residual ||r||_2/||b||_2, normwise backward error
    ||r||_inf / (||A||_inf ||u||_inf + ||b||_inf) with ||A||_inf = 8 for the
    h*h-scaled operator, error against the exact discrete solution and, with
    ref, the largest difference from the FP64 SOR result, both relative to
    the largest value."""
    import numpy as np
    sr, sb, rinf = sor.residual_f64(u, b_dev, f_dev, ctx=ctx)
    uh = u.cpu().numpy()
    out = {"rel_residual": math.sqrt(sr) / math.sqrt(sb),
           "backward_error_inf": rinf / (8.0 * float(np.max(np.abs(uh))) + b_inf),
           "max_err_vs_exact_rel": float(np.max(np.abs(uh - exact))) / scale}
    if ref is not None:
        out["max_rel_diff_vs_fp64"] = float(np.max(np.abs(uh - ref))) / float(np.max(np.abs(ref)))
    return out


def mixed_run(sor, ctx, torch, g, b, f, bits, max_outer, b_inf, exact, scale, ref, targets):
    """One timed mixed-precision solve of max_outer corrections (default inner
    count), then the same corrections one call at a time (identical
    arithmetic: every correction starts from the residual of the current
    iterate) for the backward error after each."""
    n = g.n
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sor.solve_mixed(u, b, f, g.omega, 0.0, max_outer, bits, 0, hist=True, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    final = accuracy(sor, ctx, u, b, f, b_inf, exact, scale, ref)
    steps = max(r.outer_steps, 1)
    trace = [(dt * k / steps, k, float(x)) for k, x in enumerate(r.hist)]
    u.zero_()
    bw = []
    for _ in range(r.outer_steps):
        sor.solve_mixed(u, b, f, g.omega, 0.0, 1, bits, 0, ctx=ctx)
        _, _, rinf = sor.residual_f64(u, b, f, ctx=ctx)
        bw.append(rinf / (8.0 * float(u.abs().max()) + b_inf))
    k_bw = next((k + 1 for k, x in enumerate(bw) if x <= 1e-10), None)
    inner = (max(n // 2, 1) + 5) // 6 * 6
    lups = r.outer_steps * inner * n * n
    esz = 4 if bits == 32 else 2
    # Algorithmic bytes: an inner update reads the correction and the inner
    # right-hand side and writes the correction (storage precision); a
    # correction's FP64 steps read u and h^2 f and write the inner right-hand
    # side, then read u and e and write u.
    alg = lups * 3 * esz + r.outer_steps * n * n * (2 * (16 + esz))
    out = {"secs": round(dt, 3), "outer_steps": r.outer_steps,
           "inner_iters_per_step": inner,
           "inner_glups": round(lups / dt / 1e9, 1),
           "hbm_equiv_GBs": round(alg / dt / 1e9, 1),
           "rel_history": [float(x) for x in r.hist],
           "backward_error_history": [float(f"{x:.3e}") for x in bw],
           "best_rel_residual": float(min(r.hist)),
           "secs_to": {str(t): time_to(trace, t) for t in targets},
           "secs_to_backward_error_1e-10": None if k_bw is None else
           round(dt * k_bw / steps, 3)}
    out.update(final)
    return out


def form_mixed(sor, ctx, torch):
    """The mixed-precision workload: FP64 defect correction around FP32 inner
    sweeps at 4096^2 against plain FP64 SOR, both run to their accuracy
    floors; binary16 inner storage at 1024^2, the largest side it accepts,
    beside FP32 at that side."""
    import numpy as np
    from workloads import poisson_manufactured
    targets = (1e-6, 1e-8, 1e-10)
    out = {"workload": "poisson_manufactured_4096 (seed 3), omega_opt; binary16 at "
                       "poisson_manufactured_1024 (seed 3)",
           "note": "refinement step k is timed as k/steps of the whole run (every step "
                   "does the same work); backward error = ||r||_inf / (8 ||u||_inf + "
                   "||b||_inf) in the h*h-scaled system; inner iterations per correction: "
                   "the default, n/2 rounded up to a multiple of 6; glups / inner_glups: "
                   "(inner) red-black updates per second of the whole solve (FP64: its "
                   "residual checks every 2000 iterations included); hbm_equiv_GBs: "
                   "algorithmic bytes per second (FP64 Poisson update 24 B; inner update "
                   "3 stored values; per correction 2 x (16 B + one stored value) per cell)"}
    for n in (4096, 1024):
        g = poisson_manufactured(n, seed=3)
        b = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
        f = torch.tensor(g.f, dtype=torch.float64, device="cuda")
        exact = dst_exact(n, g.bdy, g.f)
        scale = float(np.max(np.abs(exact)))
        b_inf = float(np.max(np.abs(rhs_b(n, g.bdy, g.f))))
        # Plain FP64 SOR to its floor: chunks of 2000 iterations until the
        # relative residual stops falling (three chunks without a new best).
        u64 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        trace, best, stale = [], float("inf"), 0
        t0 = time.perf_counter()
        while stale < 3 and len(trace) < 40:
            sor.solve_f64(u64, b, f, g.omega, 0.0, 2000, 2000, ctx=ctx)
            sr, sb, _ = sor.residual_f64(u64, b, f, ctx=ctx)
            rel = math.sqrt(sr) / math.sqrt(sb)
            trace.append((time.perf_counter() - t0, 2000 * (len(trace) + 1), rel))
            stale = 0 if rel < 0.99 * best else stale + 1
            best = min(best, rel)
        ref = u64.cpu().numpy()
        key = "" if n == 4096 else f"_{n}"
        its = trace[-1][1]
        rec = {"iterations": its, "secs": round(trace[-1][0], 3),
               "glups": round(its * n * n / trace[-1][0] / 1e9, 1),
               "hbm_equiv_GBs": round(24.0 * its * n * n / trace[-1][0] / 1e9, 1),
               "best_rel_residual": best,
               "secs_to": {str(t): time_to(trace, t) for t in targets}}
        rec.update(accuracy(sor, ctx, u64, b, f, b_inf, exact, scale))
        out[f"fp64_plain{key}"] = rec
        out[f"fp32_refine{key}"] = mixed_run(sor, ctx, torch, g, b, f, 32, 14 if n == 4096 else 12,
                                             b_inf, exact, scale, ref, targets)
        if n == 1024:
            out["fp16_refine_1024"] = mixed_run(sor, ctx, torch, g, b, f, 16, 30, b_inf, exact,
                                                scale, ref, targets)
        del u64, b, f
    out["fp16_refine"] = ("not run at 4096^2: binary16 inner storage is accepted for n <= "
                          "1024 only (it stalls near relative residual 1e2-1e3 from n = 1536)")
    return out


def form_batched(sor, ctx, torch, autotune=True, one_at_a_time=True):
    from workloads import batch_grids
    grids = batch_grids(512, 64, 1024, seed=4, tol=1e-8)
    us = [torch.zeros((g.n, g.n), dtype=torch.float64, device="cuda") for g in grids]
    bs = [torch.tensor(g.bdy, dtype=torch.float64, device="cuda") for g in grids]
    fs = [None if g.f is None else torch.tensor(g.f, dtype=torch.float64, device="cuda")
          for g in grids]
    out = {"workload": "512 grids, n log-uniform [64,1024] (seed 4), tol 1e-8, check every 1"}

    def timed(fn):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    specs = [sor.GridSpec(u, b, f, g.omega, 1e-8, 200000, 1)
             for u, b, f, g in zip(us, bs, fs, grids)]
    timed(lambda: sor.batch_solve_f64(specs, ctx=ctx))           # records the graph
    res, dt = timed(lambda: sor.batch_solve_f64(specs, ctx=ctx))
    lups = sum(g.n * g.n * r.iterations for g, r in zip(grids, res))
    it64 = int(sum(r.iterations for r in res))

    def rel_residuals():
        rr = []
        for u, b, f in zip(us, bs, fs):
            r2, b2, _ = sor.residual_f64(u, b, f, ctx=ctx)
            rr.append(math.sqrt(r2) / math.sqrt(b2))
        return rr
    u64 = [u.clone() for u in us]
    rel64 = rel_residuals()
    done = sorted(t for t in ctx.batch_times(len(grids)) if t == t)
    out["fp64_batched"] = {"secs": round(dt, 3), "solves_per_s": round(512 / dt, 1),
                           "glups": round(lups / dt / 1e9, 1),
                           "converged": sum(r.converged for r in res),
                           "max_rel_residual": float(f"{max(rel64):.3e}"),
                           "retire_ms_p50_max": [round(done[len(done) // 2], 1),
                                                 round(done[-1], 1)]}
    # FP32 + FP64 refinement, (a) to the accuracy the FP64 batch reached, grid
    # by grid (relative residual at most that grid's FP64 one), and (b) to a
    # correction below 1e-8.
    for key, stop in (("fp32_refine_batched_same_residual", "rel"),
                      ("fp32_refine_batched", "corr")):
        mspecs = [sor.MixedSpec(u, b, f, g.omega, r64 if stop == "rel" else 0.0,
                                1e-8 if stop == "corr" else 0.0, 50, 0)
                  for u, b, f, g, r64 in zip(us, bs, fs, grids, rel64)]
        timed(lambda: sor.batch_solve_mixed(mspecs, 32, ctx=ctx))
        res, dt = timed(lambda: sor.batch_solve_mixed(mspecs, 32, ctx=ctx))
        diff = max(float((u - v).abs().max()) / max(float(v.abs().max()), 1e-300)
                   for u, v in zip(us, u64))
        rr = rel_residuals()
        out[key] = {"secs": round(dt, 3), "solves_per_s": round(512 / dt, 1),
                    "stop": ("relative residual <= the FP64 batch's, per grid" if stop == "rel"
                             else "max |correction| < 1e-8"),
                    "converged": sum(r.converged for r in res),
                    "inner_iterations_total": int(sum(r.iterations for r in res)),
                    "grids_at_or_below_fp64_residual": sum(a <= b for a, b in zip(rr, rel64)),
                    "max_rel_residual": float(f"{max(rr):.3e}"),
                    "max_rel_diff_vs_fp64_batched": float(f"{diff:.3e}")}
    out["fp64_batched"]["iterations_total"] = it64
    del u64

    if not one_at_a_time:
        return out

    def one_at_a_time_run():
        its = 0
        for u, b, f, g in zip(us, bs, fs, grids):
            its += g.n * g.n * sor.solve_f64(u, b, f, g.omega, 1e-8, 200000, 1, ctx=ctx).iterations
        return its
    its, dt = timed(one_at_a_time_run)
    out["fp64_one_at_a_time"] = {"secs": round(dt, 3), "solves_per_s": round(512 / dt, 1),
                                 "glups": round(its / dt / 1e9, 1)}
    out["speedup_batched_vs_one_at_a_time"] = round(
        out["fp64_batched"]["solves_per_s"] / out["fp64_one_at_a_time"]["solves_per_s"], 2)

    if not autotune:
        return out
    # Autotuned tiles: one batched-throughput search per half-octave size
    # class in the batch, on a context of its own so that later forms keep
    # the default tiling.
    tctx = sor.Context(0)
    tuned = {}
    for n in sorted({g.n for g in grids}):
        c = round(2 * math.log2(n))
        if c not in tuned:
            tuned[c] = tctx.autotune_batch(64, n)
    timed(lambda: sor.batch_solve_f64(specs, ctx=tctx))          # records the graph
    res, dt = timed(lambda: sor.batch_solve_f64(specs, ctx=tctx))
    out["fp64_batched_autotuned"] = {
        "secs": round(dt, 3), "solves_per_s": round(512 / dt, 1),
        "glups": round(sum(g.n * g.n * r.iterations for g, r in zip(grids, res)) / dt / 1e9, 1),
        "converged": sum(r.converged for r in res),
        "tilings": {str(k): list(v) for k, v in sorted(tuned.items())}}
    tctx.close()
    return out


def form_tol(sor, ctx, torch, n=4096, tol=1e-8, K=10, cap=100000):
    """The benchmark grid solved to max |du| < tol (checked every K)."""
    from workloads import laplace_random_boundary
    g = laplace_random_boundary(n, seed=2)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    b = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sor.solve_f64(u, b, None, g.omega, tol, cap, K, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": f"laplace_random_boundary_{n} (seed 2), omega_opt, tol {tol}, "
                        f"check every {K}",
            "converged": bool(r.converged), "iterations": r.iterations,
            "final_max_delta": r.final_max_delta, "secs": round(dt, 3),
            "glups": round(n * n * r.iterations / dt / 1e9, 1)}


def form_paper(sor, ctx, torch, n=4096):
    """The paper's configuration: omega 0.376, north edge 1, other edges 0,
    tol 1e-5 checked every 4000 iterations, at most 50000 (Sec. 2.1, Sec. 4).
    Reports the iteration count at which the check passed, which the paper
    does not print."""
    from workloads import laplace_top_edge
    g = laplace_top_edge(n, top=1.0, tol=1e-5, max_iters=50000, check_every=4000)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    b = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sor.solve_f64(u, b, None, 0.376, g.tol, g.max_iters, g.check_every, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": f"laplace_top_edge_{n}, north 1.0, omega 0.376, tol 1e-5, "
                        "check every 4000, max 50000",
            "converged": bool(r.converged), "iterations": r.iterations,
            "final_max_delta": r.final_max_delta, "secs": round(dt, 3),
            "glups": round(n * n * r.iterations / dt / 1e9, 1)}


def form_3d(sor, ctx, torch, n=256, iters=1000, cpu=True):
    """The 3-D extension (7-point stencil on the unit cube): 256^3 interior
    cells, random boundary faces, omega_opt; a fixed iteration count for the
    update rate (kernel time from HIP events around each run of launches), then a
    solve to 1e-8 checked every 10 iterations."""
    from workloads import random_cube
    g = random_cube(21, n, with_f=False)
    b = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
    u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    sor.solve3d_f64(u, b, None, g.omega, 0.0, 20, 10, ctx=ctx)       # warm-up
    u.zero_()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sor.solve3d_f64(u, b, None, g.omega, 0.0, iters, 10, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile()
    ctx.set_profiling(False)
    lups = n ** 3 * r.iterations
    T, cx, cy, zs = ctx.tiling3d_for(n, check_every=10)
    avg_us = kern_ms * 1e3 / max(launches, 1)
    kern_s = kern_ms * 1e-3
    out = {"workload": f"laplace_random_faces_{n}^3, omega_opt",
           "kernel": f"sor3d_stream_kernel ({T} iterations per launch, grid A -> grid B)",
           "tiling": {"iters_per_launch": T, "cx": cx, "cy": cy, "zs": zs},
           "iterations": r.iterations, "secs": round(dt, 3),
           "glups": round(lups / dt / 1e9, 2),
           "avg_launch_us": round(avg_us, 2), "launches": launches,
           "glups_kernel": round(lups / kern_s / 1e9, 2),
           "hbm_equiv_GBs": round(BYTES_PER_LUP_F64 * lups / kern_s / 1e9, 1),
           "hbm_peak_GBs": HBM_PEAK_GBS}
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sor.solve3d_f64(u, b, None, g.omega, 1e-8, 100000, 10, ctx=ctx)
    torch.cuda.synchronize()
    out["tol_1e-8"] = {"converged": bool(r.converged), "iterations": r.iterations,
                       "secs": round(time.perf_counter() - t0, 3)}
    if cpu:
        import oracle
        threads = max(1, min(len(os.sched_getaffinity(0)), 16))
        iters_cpu = 200
        t0 = time.perf_counter()
        oracle.sor3d_f64(g.u0, g.bdy, None, g.omega, 0.0, iters_cpu, 10, threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"glups": round(n ** 3 * iters_cpu / dt / 1e9, 3), "cores": threads,
                             "sample": f"same {n}^3 grid, {iters_cpu} iterations, {dt:.1f} s"}
    return out


def form_variants(sor, ctx, torch, n=4096, iters=200, n_conv=128, cpu=True):
    """The Jacobi and four-colour orderings (Sec. 2.1, Sec. 3.1) and
    block-parallel SOR (Sec. 3.1; 128 x 128 blocks on the 4096^2 grid, 32 x
    32 on the 128^2 one): update rate on the 4096^2 bench grid (fixed
    iterations, kernel time from HIP events around each run of passes; 16
    algorithmic bytes per update against the 8 TB/s HBM peak), and
    iterations to 1e-8 (checked every 10) on a 128^2 grid next to red-black,
    each at its best omega (Jacobi: 1; block-parallel: 1.45, the best of a
    0.05 grid on the oracle, since it diverges from about 1.48 on).  All run
    their blocked passes of several iterations each (Jacobi 8, four-colour
    5, block-parallel 5 by default)."""
    from workloads import laplace_random_boundary
    g = laplace_random_boundary(n)
    b = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
    out = {"workload": f"laplace_random_boundary_{n}, {iters} iterations; "
                       f"laplace_random_boundary_{n_conv} to 1e-8"}
    bp_big, bp_small, bp_omega = 128, 32, 1.45

    def solve(name, u, bdy, omega, tol, it):
        if name == "block_parallel":
            blk = bp_big if u.shape[0] == n else bp_small
            return sor.solve_blockpar_f64(u, bdy, blk, blk, None, omega, tol, it, 10, ctx=ctx)
        ordering = {"jacobi": sor.ORDER_JACOBI, "four_colour": sor.ORDER_FOUR_COLOUR,
                    "red_black": sor.ORDER_RED_BLACK}[name]
        return sor.solve_variant_f64(ordering, u, bdy, None, omega, tol, it, 10, ctx=ctx)

    rate_cases = (("jacobi", 1.0), ("four_colour", g.omega), ("block_parallel", 1.0))
    for name, omega in rate_cases:
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        solve(name, u, b, omega, 0.0, 10)
        u.zero_()
        ctx.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = solve(name, u, b, omega, 0.0, iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kern_ms, launches = ctx.profile()
        ctx.set_profiling(False)
        it_us = kern_ms * 1e3 / max(r.iterations, 1)
        out[name] = {"glups": round(n * n * r.iterations / dt / 1e9, 1),
                     "launches": launches,
                     "us_per_iteration": round(it_us, 2),
                     "glups_kernel": round(n * n / (it_us * 1e-6) / 1e9, 1),
                     "hbm_equiv_GBs": round(BYTES_PER_LUP_F64 * n * n / (it_us * 1e-6) / 1e9, 1),
                     "hbm_frac": round(BYTES_PER_LUP_F64 * n * n / (it_us * 1e-6) / 1e9
                                       / HBM_PEAK_GBS, 3)}
    out["block_parallel"]["blocks"] = [bp_big, bp_big]
    out["block_parallel"]["tiling"] = list(ctx.get_variant_tiling(sor.ORDER_BLOCK_PARALLEL))
    gc = laplace_random_boundary(n_conv)
    bc = torch.tensor(gc.bdy, dtype=torch.float64, device="cuda")
    conv = {}
    for name, omega in (("red_black", gc.omega), ("four_colour", gc.omega), ("jacobi", 1.0),
                        ("block_parallel", bp_omega)):
        u = torch.zeros((n_conv, n_conv), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = solve(name, u, bc, omega, 1e-8, 1000000)
        torch.cuda.synchronize()
        conv[name] = {"converged": bool(r.converged), "iterations": r.iterations,
                      "secs": round(time.perf_counter() - t0, 3), "omega": round(omega, 4)}
    conv["block_parallel"]["blocks"] = [bp_small, bp_small]
    out["to_1e-8"] = conv
    if cpu:
        import oracle
        iters_cpu = 8
        for name, omega in rate_cases:
            t0 = time.perf_counter()
            if name == "block_parallel":
                oracle.blockpar_f64(g.u0, g.bdy, None, omega, bp_big, bp_big, 0.0, iters_cpu, 10)
            else:
                ordering = oracle.ORDER_JACOBI if name == "jacobi" else oracle.ORDER_FOUR_COLOUR
                oracle.variant_f64(ordering, g.u0, g.bdy, None, omega, 0.0, iters_cpu, 10)
            dt = time.perf_counter() - t0
            out[name]["cpu_oracle"] = {"glups": round(n * n * iters_cpu / dt / 1e9, 3),
                                       "cores": 1,
                                       "sample": f"same {n}^2 grid, {iters_cpu} iterations, "
                                                 f"single thread, {dt:.1f} s"}
    return out


def form_control(sor, ctx, torch, n=8192, iters=300, K=10):
    """8192^2 FP64 Laplace (two 537 MB grids, beyond the 256 MB Infinity
    Cache), fixed iterations: GLUP/s with the automatic tiling."""
    from workloads import laplace_random_boundary
    g = laplace_random_boundary(n)
    b = torch.tensor(g.bdy, dtype=torch.float64, device="cuda")
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    sor.solve_f64(u, b, None, g.omega, 0.0, 2 * K, K, ctx=ctx)
    u.zero_()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sor.solve_f64(u, b, None, g.omega, 0.0, iters, K, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.profile()
    ctx.set_profiling(False)
    T, seg = ctx.tiling_for(64, n)
    lups = float(n) * n * r.iterations
    return {"workload": f"laplace_random_boundary_{n}, omega_opt, {iters} iterations, "
                        f"check every {K}",
            "tiling": {"iters_per_pass": T, "seg_rows": seg},
            "glups": round(lups / dt / 1e9, 1),
            "glups_kernel": round(lups / (kern_ms * 1e-3) / 1e9, 1),
            "avg_launch_us": round(kern_ms * 1e3 / max(launches, 1), 2),
            "bandwidth_equiv_GBs": round(BYTES_PER_LUP_F64 * lups / (kern_ms * 1e-3) / 1e9, 1)}


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def form_serving(sor, ctx, torch, count, burst):
    import numpy as np
    from workloads import ServingStream
    tol = 1e-8
    # n inner iterations per correction (rounded up to a multiple of the
    # persistent kernel's depth, 6): fewer, longer corrections than the
    # library default (about n/2) pay off here, since every correction's
    # phase changes meet the time-slice boundaries; measured (at depth 4)
    # 113-122 solves/s against 99-110 for the default and 93 for 2n.
    inner = lambda n: (n + 5) // 6 * 6
    srv = sor.Server(0, inner_bits=32, hbm_budget=64 << 30, max_slots=128, slice_ms=2.0)
    try:
        # Saturated rate: a closed-loop burst of `burst` requests.
        probe = ServingStream(burst, 1.0, seed=55)
        t0 = time.perf_counter()
        ts = []
        for k in range(burst):
            n, bdy, f = probe.request(k)
            ts.append(srv.submit(bdy, f, None, 0.0, tol, 0.0, 50, inner(n)))
        for t in ts:
            while srv.poll(t, wait_ms=50.0) is None:
                pass
        sat = burst / (time.perf_counter() - t0)
        rate = 0.7 * sat
        stream = ServingStream(count, rate, seed=5)
        lat, bad = [], 0
        pending = {}
        t0 = time.perf_counter()
        k = 0
        while k < count or pending:
            now = time.perf_counter() - t0
            while k < count and stream.arrivals[k] <= now:
                n, bdy, f = stream.request(k)
                t_sub = time.perf_counter() - t0
                pending[srv.submit(bdy, f, None, 0.0, tol, 0.0, 50, inner(n))] = (
                    stream.arrivals[k], t_sub)
                k += 1
            for t in list(pending):
                c = srv.poll(t)
                if c is not None:
                    arr, t_sub = pending.pop(t)
                    lat.append((c.done_s - c.submit_s) + (t_sub - arr))
                    bad += c.status != sor.OK
            time.sleep(0.0005)
        makespan = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    served = {"requests": count, "rate_per_s": round(rate, 2),
              "saturated_solves_per_s": round(sat, 2),
              "solves_per_s": round(count / makespan, 2),
              "p50_latency_ms": round(1e3 * percentile(lat, 50), 2),
              "p99_latency_ms": round(1e3 * percentile(lat, 99), 2),
              "not_converged": bad, "launches": st["launches"]}
    # Baseline: the same arrivals through one-at-a-time plain FP64 (FIFO),
    # relative residual checked every max(200, n) iterations.
    lat0, its_total = [], 0
    t0 = time.perf_counter()
    for k in range(count):
        n, bdy, f = stream.request(k)
        now = time.perf_counter() - t0
        if stream.arrivals[k] > now:
            time.sleep(stream.arrivals[k] - now)
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        b = torch.tensor(bdy, dtype=torch.float64, device="cuda")
        ff = torch.tensor(f, dtype=torch.float64, device="cuda")
        its, rel = fp64_to_residual(sor, ctx, u, b, ff, sor.omega_opt(n), tol,
                                    max(200, n), 40 * n)
        _ = u.cpu()
        lat0.append(time.perf_counter() - t0 - stream.arrivals[k])
    span0 = time.perf_counter() - t0
    base = {"solves_per_s": round(count / span0, 2),
            "p50_latency_ms": round(1e3 * percentile(lat0, 50), 2),
            "p99_latency_ms": round(1e3 * percentile(lat0, 99), 2)}
    return {"workload": f"{count} requests, n log-uniform [128,2048] (seed 5), "
                        "rel residual 1e-8, FP32 inner (n iterations per correction) + "
                        "FP64 refinement, HBM budget 64 GiB, 128 slots, 2 ms slices",
            "served": served, "fp64_one_at_a_time_same_arrivals": base,
            "speedup_solves_per_s": round(served["solves_per_s"] / base["solves_per_s"], 2),
            "p99_ratio_baseline_over_served": round(base["p99_latency_ms"] / served["p99_latency_ms"], 2)}


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
    ap.add_argument("--forms", default="tol,paper,control,mixed,batched,3d,variants,serving",
                    help="comma list of extra forms to measure, or 'none'")
    ap.add_argument("--no-batch-extras", action="store_true",
                    help="batched form: skip the one-at-a-time and autotuned legs")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-burst", type=int, default=80)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one device-to-device copy of this "
                         "many MiB (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(a grid would shard into row slabs with 2T-row ghost zones exchanged "
              "once per pass); run with --gpus 1", file=sys.stderr)
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
    T, seg = ctx.tiling_for(64, n)
    print(f"[bench] n={n} iters={iters} K={K} tiling T={T} seg_rows={seg}",
          file=sys.stderr, flush=True)

    def step():
        u.zero_()                     # the workload's interior starts at 0
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
    lups = float(n) * n * iters * args.steps          # in the timed kernels
    achieved = FLOPS_PER_LUP_F64 * lups / (kern_ms / 1e3) / 1e12
    issue = INSTR_PER_LUP_F64 * lups / (kern_ms / 1e3) / 1e12
    alg_bytes = BYTES_PER_LUP_F64 * n * n * T         # one full-depth pass
    traffic = measured_traffic(n, T, seg)
    hbm_meas = None if traffic is None else traffic / avg_launch_s / 1e9
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
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4),
                     "traffic": traffic,
                     "kernel": f"blocked_pass_kernel<f64,T={T},laplace>",
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "launches": launches,
                     "alg_flops_per_launch": FLOPS_PER_LUP_F64 * n * n * T,
                     "valu_issue_Tinstr_s": round(issue, 3),
                     "valu_issue_peak_Tinstr_s": round(FP64_VALU_ISSUE_TIPS, 2),
                     "valu_issue_frac": round(issue / FP64_VALU_ISSUE_TIPS, 4),
                     "hbm_measured_GBs": None if hbm_meas is None else round(hbm_meas, 1),
                     "hbm_measured_frac": None if hbm_meas is None else
                     round(hbm_meas / HBM_PEAK_GBS, 4),
                     "hbm_equiv_GBs": round(BYTES_PER_LUP_F64 * lups / (kern_ms / 1e3) / 1e9, 1),
                     "hbm_peak_GBs": HBM_PEAK_GBS,
                     "alg_bytes_per_launch": alg_bytes},
        "bandwidth_equiv_GBs": round(glups * BYTES_PER_LUP_F64, 1),
    }
    if not args.copy_probe_mib:
        line["roofline"]["hbm_achievable_copy_GBs"] = copy_bandwidth(torch)
    forms = [] if args.forms == "none" else args.forms.split(",")
    line["forms"] = {}
    if "tol" in forms:
        print("[bench] form: 4096^2 to tolerance", file=sys.stderr, flush=True)
        line["forms"]["tol"] = form_tol(sor, ctx, torch)
    if "paper" in forms:
        print("[bench] form: the paper's configuration", file=sys.stderr, flush=True)
        line["forms"]["paper"] = form_paper(sor, ctx, torch)
    if "mixed" in forms:
        print("[bench] form: mixed precision 4096^2", file=sys.stderr, flush=True)
        line["forms"]["mixed"] = form_mixed(sor, ctx, torch)
    if "batched" in forms:
        print("[bench] form: batched 512 grids", file=sys.stderr, flush=True)
        line["forms"]["batched"] = form_batched(sor, ctx, torch,
                                                autotune=not args.no_batch_extras,
                                                one_at_a_time=not args.no_batch_extras)
    if "control" in forms:
        print("[bench] form: 8192^2 control", file=sys.stderr, flush=True)
        line["forms"]["control_8192"] = form_control(sor, ctx, torch)
    if "variants" in forms:
        print("[bench] form: Jacobi and four-colour orderings", file=sys.stderr, flush=True)
        line["forms"]["variants"] = form_variants(sor, ctx, torch,
                                                  cpu=not args.no_cpu_baseline)
    if "3d" in forms:
        print("[bench] form: 3-D 256^3", file=sys.stderr, flush=True)
        line["forms"]["3d"] = form_3d(sor, ctx, torch, cpu=not args.no_cpu_baseline)
    if "serving" in forms:
        print("[bench] form: serving", file=sys.stderr, flush=True)
        line["forms"]["serving"] = form_serving(sor, ctx, torch, args.serve_requests,
                                                args.serve_burst)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
