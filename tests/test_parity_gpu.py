"""GPU parity: the HIP path against the CPU oracle on identical seeded inputs.

FP64 and FP32 plain solves must agree with the oracle bit for bit (same
update expression and roundings, the quarter-difference fused on both sides,
exact max) -- both the final grid and every
iteration's max change -- and stop at the same iteration.  Mixed precision
must agree bit for bit at a fixed number of corrections.  The residual must
agree bit for bit per cell; its sums (different summation order) to 1e-12.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import (laplace_random_boundary, laplace_top_edge, omega_opt,
                       poisson_manufactured, random_small)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sor():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1401_0763_amd as m
    return m


@pytest.fixture()
def ctx(sor):
    c = sor.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dtype,
                                               device="cuda")


def run_gpu(sor, ctx, g, tol, iters, K, dtype=torch.float64, hist=True):
    u = dev(g.u0, dtype)
    fn = sor.solve_f64 if dtype == torch.float64 else sor.solve_f32
    res = fn(u, dev(g.bdy, dtype), dev(g.f, dtype), g.omega, tol, iters, K,
             hist=hist, ctx=ctx)
    return res, u.cpu().numpy()


def assert_bitwise(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    if not np.array_equal(a.view(np.uint64 if a.dtype == np.float64 else np.uint32),
                          b.view(np.uint64 if b.dtype == np.float64 else np.uint32)):
        diff = np.abs(a.astype(np.float64) - b.astype(np.float64))
        k = np.unravel_index(np.argmax(diff), diff.shape)
        raise AssertionError(f"{what}: {np.count_nonzero(diff)} differ; max {diff.max()} at {k}")


# ---------------------------------------------------------------------------
# FP64, fixed iteration count, many tilings
# ---------------------------------------------------------------------------

TILINGS = [(1, 8), (2, 16), (3, 8), (4, 64), (5, 40), (6, 32), (6, 8), (4, 192), (5, 128),
           (6, 128), (7, 40), (7, 94), (8, 16), (8, 102)]


@pytest.mark.parametrize("n,with_f,iters", [
    (1, True, 7), (2, False, 9), (3, True, 13), (17, True, 31), (64, False, 40),
    (100, True, 37), (255, True, 50), (300, False, 23)])
def test_f64_fixed_iterations_bitwise_all_tilings(sor, ctx, n, with_f, iters):
    g = random_small(1000 + n, n, with_f=with_f, nonzero_u0=True)
    ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 0.0, iters, 1, hist=True)
    for T, seg in TILINGS:
        _say(f"f64 n={n} f={with_f} iters={iters} T={T} seg={seg}")
        ctx.set_kernel(sor.KERNEL_BLOCKED)
        ctx.set_tiling(64, T, seg)
        res, u = run_gpu(sor, ctx, g, 0.0, iters, 1)
        assert res.status == sor.NOT_CONVERGED and res.iterations == iters
        assert_bitwise(u, ref.u, f"u n={n} T={T} seg={seg}")
        assert_bitwise(np.array(res.hist), ref.mhist, f"hist n={n} T={T}")
    _say(f"f64 n={n} simple kernel")
    ctx.set_kernel(sor.KERNEL_SIMPLE)
    res, u = run_gpu(sor, ctx, g, 0.0, iters, 1)
    assert_bitwise(u, ref.u, f"u n={n} simple")
    assert_bitwise(np.array(res.hist), ref.mhist, f"hist n={n} simple")


def test_f64_laplace_top_edge_to_convergence_k1(sor, ctx):
    """256x256 Laplace, north = 100, omega_opt, tol 1e-6 checked every iteration."""
    g = laplace_top_edge(256)
    ref = oracle.sor_f64(g.u0, g.bdy, None, g.omega, g.tol, g.max_iters, 1, hist=True)
    assert ref.status == oracle.OK
    for T, seg in [(4, 64), (3, 32), (6, 256)]:
        _say(f"top edge 256 T={T} seg={seg}")
        ctx.set_tiling(64, T, seg)
        res, u = run_gpu(sor, ctx, g, g.tol, g.max_iters, 1)
        assert res.status == sor.OK and res.converged
        assert res.iterations == ref.iterations
        assert res.final_max_delta == ref.final_max_delta
        assert_bitwise(u, ref.u, "u")
        assert_bitwise(np.array(res.hist), ref.mhist, "hist")


@pytest.mark.parametrize("K,T", [(10, 4), (7, 3), (1, 6), (5, 6), (3, 2), (4, 5), (10, 5),
                                 (10, 7), (3, 7), (10, 8), (5, 8)])
def test_f64_check_cadence_and_rollback(sor, ctx, K, T):
    """Stops at the first checked iteration below tol, also inside a pass."""
    n = 48
    g = random_small(7, n, with_f=True)
    full = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 0.0, 600, 1, hist=True)
    for tol in (1e-3, 1e-6, 1e-9):
        ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, tol, 600, K)
        _say(f"cadence K={K} T={T} tol={tol} ref_it={ref.iterations}")
        ctx.set_tiling(64, T, 16)
        res, u = run_gpu(sor, ctx, g, tol, 600, K)
        assert res.status == ref.status
        assert res.iterations == ref.iterations
        assert res.final_max_delta == ref.final_max_delta
        assert_bitwise(u, ref.u, "u")
        assert_bitwise(np.array(res.hist), full.mhist[: ref.iterations], "hist")


@pytest.mark.parametrize("max_iters", [1, 5, 11, 1030])
def test_f64_iteration_limit_not_multiple_of_pass(sor, ctx, max_iters):
    n = 33
    g = random_small(8, n, with_f=False)
    ref = oracle.sor_f64(g.u0, g.bdy, None, g.omega, 0.0, max_iters, 4)
    ctx.set_tiling(64, 6, 8)
    res, u = run_gpu(sor, ctx, g, 0.0, max_iters, 4, hist=False)
    assert res.status == sor.NOT_CONVERGED and res.iterations == max_iters
    assert res.final_max_delta == ref.final_max_delta
    assert_bitwise(u, ref.u, "u")


def test_f64_underrelaxation_paper_omega(sor, ctx):
    """The paper's omega = 0.376, north edge 1.0, others 0 (Sec. 2.1, 3.4)."""
    n = 96
    bdy = np.zeros(4 * n)
    bdy[:n] = 1.0
    ref = oracle.sor_f64(np.zeros((n, n)), bdy, None, 0.376, 1e-5, 400, 40, hist=True)
    from workloads import Grid
    g = Grid(n, np.zeros((n, n)), bdy, None, 0.376)
    ctx.set_tiling(64, 4, 64)
    res, u = run_gpu(sor, ctx, g, 1e-5, 400, 40)
    assert res.iterations == ref.iterations and res.status == ref.status
    assert_bitwise(u, ref.u, "u")


def test_f64_nonfinite_boundary_reported(sor, ctx):
    n = 20
    g = random_small(9, n, with_f=False)
    g.bdy[5] = np.nan
    ref = oracle.sor_f64(g.u0, g.bdy, None, g.omega, 1e-6, 100, 1)
    assert ref.status == oracle.ENONFINITE
    for kernel in (sor.KERNEL_BLOCKED, sor.KERNEL_SIMPLE):
        ctx.set_kernel(kernel)
        res, _ = run_gpu(sor, ctx, g, 1e-6, 100, 1, hist=False)
        assert res.status == sor.ENONFINITE


@pytest.mark.parametrize("bits,n,scale,first_bad", [
    (64, 130, 0.15, 6), (64, 130, 0.2, 3), (64, 37, 0.25, 2),
    (32, 130, 0.15, 6), (32, 37, 0.25, 2)])
def test_overflow_during_solve_reported(sor, ctx, bits, n, scale, first_bad):
    """Finite inputs whose iterates overflow: with a uniform boundary near a
    fraction of the largest finite value, over-relaxation overshoots and a
    neighbour sum leaves the finite range after a few iterations, between two
    checks (K = 10).  Every solve must stop with ENONFINITE by the end of the
    pass in which the oracle finds the first infinite change, with the same
    changes up to and including that iteration (the infinite one included)."""
    dtype = torch.float64 if bits == 64 else torch.float32
    top = float(np.finfo(np.float64 if bits == 64 else np.float32).max)
    v = float(np.float32(scale * top)) if bits == 32 else scale * top
    from workloads import Grid
    g = Grid(n, np.zeros((n, n)), np.full(4 * n, v), None, omega_opt(n))
    fn = oracle.sor_f64 if bits == 64 else oracle.sor_f32
    ref = fn(g.u0, g.bdy, None, g.omega, 0.0, 100, 10, hist=True)
    assert ref.status == oracle.ENONFINITE and ref.iterations == first_bad
    assert math.isinf(ref.mhist[-1])
    for T, seg in [(1, 8), (4, 64), (7, 94), (8, 16), (0, 0)]:
        _say(f"overflow bits={bits} n={n} scale={scale} T={T} seg={seg}")
        if T:
            ctx.set_kernel(sor.KERNEL_BLOCKED)
            ctx.set_tiling(bits, T, seg)
        else:
            ctx.set_kernel(sor.KERNEL_SIMPLE)
        res, _ = run_gpu(sor, ctx, g, 0.0, 100, 10, dtype=dtype)
        assert res.status == sor.ENONFINITE and not res.converged, (T, res)
        span = T if T else 1
        assert first_bad <= res.iterations < first_bad + span, (T, res.iterations)
        assert_bitwise(np.array(res.hist[:first_bad]), ref.mhist,
                       f"changes up to the overflow, T={T}")


def test_invalid_arguments_rejected(sor, ctx):
    n = 8
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    b = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    for kw in (dict(omega=0.0), dict(omega=2.0), dict(tol=float("nan")),
               dict(max_iters=0), dict(check_every=0)):
        args = dict(omega=1.5, tol=1e-6, max_iters=10, check_every=1)
        args.update(kw)
        with pytest.raises(sor.SorError) as e:
            sor.solve_f64(u, b, None, ctx=ctx, **args)
        assert e.value.status == sor.EINVAL
    # host pointers are refused by the library, not dereferenced
    import ctypes
    hu = np.zeros((n, n))
    hb = np.zeros(4 * n)
    res = sor._Result()
    st = ctx.lib.sor_solve_f64(ctx.handle, ctypes.c_void_p(hu.ctypes.data),
                               ctypes.c_void_p(hb.ctypes.data), None, n, 1.5, 1e-6,
                               10, 1, None, ctypes.byref(res), None)
    assert st == sor.EINVAL
    # empty and oversized grids are refused before anything is read
    for bad_n in (0, -3, 65537):
        st = ctx.lib.sor_solve_f64(ctx.handle, ctypes.c_void_p(u.data_ptr()),
                                   ctypes.c_void_p(b.data_ptr()), None, bad_n, 1.5, 1e-6,
                                   10, 1, None, ctypes.byref(res), None)
        assert st == sor.EINVAL, bad_n
        for fn in (ctx.lib.sor_solve3d_f64,):
            assert fn(ctx.handle, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                      None, bad_n if bad_n != 65537 else 1025, 1.5, 1e-6, 10, 1, None,
                      ctypes.byref(res), None) == sor.EINVAL, bad_n
        for ordering in (1, 2):
            assert ctx.lib.sor_solve_variant_f64(
                ctx.handle, ordering, ctypes.c_void_p(u.data_ptr()),
                ctypes.c_void_p(b.data_ptr()), None, bad_n, 1.0, 1e-6, 10, 1, None,
                ctypes.byref(res), None) == sor.EINVAL, (ordering, bad_n)
    with pytest.raises(sor.SorError):
        ctx.set_tiling(64, 9, 64)
    with pytest.raises(sor.SorError):
        ctx.set_tiling(64, 4, 7)


# ---------------------------------------------------------------------------
# FP32 storage
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,with_f", [(1, True), (5, False), (77, True), (260, True)])
def test_f32_fixed_iterations_bitwise(sor, ctx, n, with_f):
    g = random_small(2000 + n, n, with_f=with_f, nonzero_u0=True)
    g.u0 = g.u0.astype(np.float32).astype(np.float64)
    g.bdy = g.bdy.astype(np.float32).astype(np.float64)
    if g.f is not None:
        g.f = g.f.astype(np.float32).astype(np.float64)
    ref = oracle.sor_f32(g.u0, g.bdy, g.f, g.omega, 0.0, 29, 1, hist=True)
    for T, seg in [(1, 8), (4, 64), (6, 16), (4, 96), (7, 64), (8, 32)]:
        _say(f"f32 n={n} T={T} seg={seg}")
        ctx.set_kernel(sor.KERNEL_BLOCKED)
        ctx.set_tiling(32, T, seg)
        res, u = run_gpu(sor, ctx, g, 0.0, 29, 1, dtype=torch.float32)
        assert_bitwise(u, ref.u, f"u f32 n={n} T={T}")
        assert_bitwise(np.array(res.hist), ref.mhist, f"hist f32 n={n} T={T}")
    ctx.set_kernel(sor.KERNEL_SIMPLE)
    res, u = run_gpu(sor, ctx, g, 0.0, 29, 1, dtype=torch.float32)
    assert_bitwise(u, ref.u, f"u f32 n={n} simple")


def test_f32_convergence_iteration_matches(sor, ctx):
    g = random_small(31, 90, with_f=True)
    g.bdy = g.bdy.astype(np.float32).astype(np.float64)
    g.f = g.f.astype(np.float32).astype(np.float64)
    ref = oracle.sor_f32(g.u0, g.bdy, g.f, g.omega, 1e-3, 5000, 3)
    assert ref.status == oracle.OK
    ctx.set_tiling(32, 4, 32)
    res, u = run_gpu(sor, ctx, g, 1e-3, 5000, 3, dtype=torch.float32, hist=False)
    assert res.iterations == ref.iterations and res.converged
    assert_bitwise(u, ref.u, "u")


# ---------------------------------------------------------------------------
# FP64 residual and mixed precision
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,with_f", [(1, True), (9, False), (300, True)])
def test_residual_bitwise_cells_and_sums(sor, ctx, n, with_f):
    g = random_small(3000 + n, n, with_f=with_f, nonzero_u0=True)
    r_ref, sr, sb, mr = oracle.residual_f64(g.u0, g.bdy, g.f)
    r = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    s = sor.residual_f64(dev(g.u0), dev(g.bdy), dev(g.f), r=r, ctx=ctx)
    assert_bitwise(r.cpu().numpy(), r_ref, "r")
    assert abs(s[0] - sr) <= 1e-12 * sr and abs(s[1] - sb) <= 1e-12 * sb
    assert s[2] == mr


@pytest.mark.parametrize("bits,n,outer", [(32, 63, 3), (32, 200, 2), (16, 63, 3), (16, 130, 2)])
def test_mixed_fixed_outer_steps_bitwise(sor, ctx, bits, n, outer):
    g = poisson_manufactured(n, seed=40 + n)
    inner = 2 * n
    ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, outer, bits, inner)
    for T, seg in [(4, 64), (3, 16), (8, 48)]:
        _say(f"mixed bits={bits} n={n} T={T}")
        ctx.set_kernel(sor.KERNEL_BLOCKED)
        ctx.set_tiling(bits, T, seg)
        u = dev(g.u0)
        res = sor.solve_mixed(u, dev(g.bdy), dev(g.f), g.omega, 0.0, outer, bits,
                              inner, hist=True, ctx=ctx)
        assert res.outer_steps == outer == ref.outer_steps
        assert_bitwise(u.cpu().numpy(), ref.u, f"u mixed{bits} n={n}")
        np.testing.assert_allclose(res.hist, ref.relhist, rtol=1e-10)


@pytest.mark.parametrize("bits,tol", [(32, 1e-12), (16, 1e-10)])
def test_mixed_reaches_tolerance_like_oracle(sor, ctx, bits, tol):
    n = 127
    g = poisson_manufactured(n, seed=77)
    ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, tol, 40, bits, 2 * n)
    assert ref.converged
    u = dev(g.u0)
    res = sor.solve_mixed(u, dev(g.bdy), dev(g.f), g.omega, tol, 40, bits, 2 * n,
                          ctx=ctx)
    assert res.converged and res.outer_steps == ref.outer_steps
    assert res.rel_residual <= tol
    assert_bitwise(u.cpu().numpy(), ref.u, "u")


# ---------------------------------------------------------------------------
# The full-size workload, in the configuration the benchmark times
# ---------------------------------------------------------------------------

def test_f64_full_size_4096_fixed_iterations_bitwise(sor, ctx):
    """4096^2 Laplace, random boundary in [0, 100], omega_opt, 200 iterations,
    checked every 10: whole grid and per-iteration changes bit for bit."""
    g = laplace_random_boundary(4096, seed=2)
    iters = 200
    _say("4096 oracle (threads)")
    ref = oracle.sor_f64(g.u0, g.bdy, None, g.omega, 0.0, iters, 10,
                         threads=min(16, os.cpu_count() or 1), hist=True)
    _say("4096 gpu")
    res, u = run_gpu(sor, ctx, g, 0.0, iters, 10)
    assert res.iterations == iters
    assert_bitwise(u, ref.u, "u 4096")
    assert_bitwise(np.array(res.hist), ref.mhist, "hist 4096")


# ---------------------------------------------------------------------------
# Subnormal values: the fused quarter-difference and relaxation step round
# exactly like the oracle's fma also where 0.25*s or the result is subnormal
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [5e-308, 3e-309])
def test_f64_subnormal_range_bitwise(sor, ctx, scale):
    n = 70
    rng = np.random.default_rng(31)
    bdy = rng.uniform(0.0, 1.0, size=4 * n) * scale
    u0 = rng.uniform(0.0, 1.0, size=(n, n)) * scale
    f = rng.standard_normal((n, n)) * scale * 1e3
    for with_f in (False, True):
        ff = f if with_f else None
        ref = oracle.sor_f64(u0, bdy, ff, 1.7, 0.0, 40, 1, hist=True)
        assert np.any((ref.u != 0) & (np.abs(ref.u) < 2.2250738585072014e-308))
        for T, seg in ((6, 32), (5, 40), (2, 16), (7, 40), (8, 32)):
            _say(f"subnormal f64 scale={scale} f={with_f} T={T}")
            ctx.set_tiling(64, T, seg)
            u = dev(u0)
            res = sor.solve_f64(u, dev(bdy), dev(ff), 1.7, 0.0, 40, 1, hist=True, ctx=ctx)
            assert_bitwise(u.cpu().numpy(), ref.u, f"u scale={scale} T={T}")
            assert_bitwise(np.array(res.hist), ref.mhist, f"hist scale={scale} T={T}")


def test_f32_subnormal_range_bitwise(sor, ctx):
    n = 70
    rng = np.random.default_rng(32)
    bdy = (rng.uniform(0.0, 1.0, size=4 * n) * 3e-38).astype(np.float32)
    u0 = (rng.uniform(0.0, 1.0, size=(n, n)) * 3e-38).astype(np.float32)
    ref = oracle.sor_f32(u0, bdy, None, 1.7, 0.0, 40, 1, hist=True)
    assert np.any((ref.u != 0) & (np.abs(ref.u) < np.finfo(np.float32).tiny))
    u = dev(u0, torch.float32)
    res = sor.solve_f32(u, dev(bdy, torch.float32), None, 1.7, 0.0, 40, 1, hist=True, ctx=ctx)
    assert_bitwise(u.cpu().numpy(), ref.u, "f32 subnormal u")


def test_3d_and_orderings_subnormal_range_bitwise(sor, ctx):
    n = 20
    rng = np.random.default_rng(33)
    faces = rng.uniform(0.0, 1.0, size=(6, n, n)) * 5e-308
    u0 = rng.uniform(0.0, 1.0, size=(n, n, n)) * 5e-308
    ref = oracle.sor3d_f64(u0, faces, None, 1.6, 0.0, 30, 1)
    for K in (1, 2):
        u = dev(u0)
        sor.solve3d_f64(u, dev(faces), None, 1.6, 0.0, 30, K, ctx=ctx)
        assert_bitwise(u.cpu().numpy(), ref.u, f"3-D subnormal K={K}")
    bdy = rng.uniform(0.0, 1.0, size=4 * 50) * 5e-308
    u2 = rng.uniform(0.0, 1.0, size=(50, 50)) * 5e-308
    for ordering in (1, 2):
        ref = oracle.variant_f64(ordering, u2, bdy, None, 1.3, 0.0, 25, 1)
        u = dev(u2)
        sor.solve_variant_f64(ordering, u, dev(bdy), None, 1.3, 0.0, 25, 1, ctx=ctx)
        assert_bitwise(u.cpu().numpy(), ref.u, f"ordering {ordering} subnormal")


def test_automatic_depth(sor):
    """A fresh context chooses the depth per solve (reported as 0): 7 for FP64
    and FP32, Laplace and Poisson problems alike.  Setting a depth ends the
    automatic choice."""
    c = sor.Context(0)
    try:
        assert c.get_tiling(64) == (0, 0)
        assert c.tiling_for(64, 4096)[0] == 7
        assert c.tiling_for(64, 4096, has_rhs=True)[0] == 7
        assert c.tiling_for(32, 4096)[0] == 7
        assert c.tiling_for(32, 4096, has_rhs=True)[0] == 7
        c.set_tiling(64, 0, 64)
        assert c.get_tiling(64) == (0, 64) and c.tiling_for(64, 4096) == (7, 64)
        c.set_tiling(64, 6, 0)
        assert c.get_tiling(64) == (6, 64) and c.tiling_for(64, 4096, True) == (6, 64)
        assert c.tiling_for(64, 4096)[0] == 6
    finally:
        c.close()


def test_profiling_counts_working_passes(sor, ctx):
    """Profiling times runs of passes; the launch count is the number of
    passes that did work, and profiling changes no result."""
    n = 200
    g = random_small(61, n, with_f=True)
    ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 0.0, 100, 10)
    ctx.set_tiling(64, 7, 0)
    ctx.set_profiling(True)
    res, u = run_gpu(sor, ctx, g, 0.0, 100, 10, hist=False)
    ms, launches = ctx.profile()
    ctx.set_profiling(False)
    assert res.passes == launches == 15          # 14 passes of 7, then one of 2
    assert ms > 0.0
    assert_bitwise(u, ref.u, "u with profiling")
    # A stop inside a pass: the passes queued after it exit at once and are
    # not counted; the re-run that rebuilds the stop iterate is not timed.
    ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 1e-6, 100000, 3)
    ctx.set_profiling(True)
    res, u = run_gpu(sor, ctx, g, 1e-6, 100000, 3, hist=False)
    ms, launches = ctx.profile()
    ctx.set_profiling(False)
    assert res.status == sor.OK and res.iterations == ref.iterations
    assert launches == -(-res.iterations // 7)
    assert_bitwise(u, ref.u, "u with profiling, stopped")
