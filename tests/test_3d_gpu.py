"""GPU parity of the 3-D path (7-point red-black SOR on the unit cube, the
extension Sec. 5 of Mittal 2014 names as future work) against the 3-D oracle
on identical seeded inputs: the final grid and every iteration's largest
change agree bit for bit (same update expression and sum order, no
contraction, exact maxima), and a solve to tolerance stops at the same
checked iteration."""
import math
import sys

import numpy as np
import pytest

import oracle
from workloads import omega_opt, random_cube

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


def dev(a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                               device="cuda")


def assert_bitwise(a, b, what):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if not np.array_equal(a.view(np.uint64), b.view(np.uint64)):
        diff = np.abs(a - b)
        k = np.unravel_index(np.argmax(diff), diff.shape)
        raise AssertionError(f"{what}: {np.count_nonzero(diff)} differ; max {diff.max()} at {k}")


def run3(sor, ctx, g, tol, iters, K, hist=True):
    u = dev(g.u0)
    res = sor.solve3d_f64(u, dev(g.bdy), dev(g.f), g.omega, tol, iters, K, hist=hist, ctx=ctx)
    return res, u.cpu().numpy()


# Streaming-kernel set-ups (iterations per launch, core cx, cy, zs; 0 =
# automatic): ragged strips, bands and z-ranges, one-plane ranges, the widest
# strips, one and two iterations per launch.  Two iterations per launch need
# an even check_every; the odd iteration counts below end with a
# one-iteration launch.
TILINGS3 = [(0, 0, 0, 0), (1, 3, 2, 2), (2, 3, 2, 2), (1, 4, 3, 3), (2, 4, 3, 3),
            (1, 7, 5, 1), (2, 9, 4, 1), (1, 124, 0, 0), (2, 120, 0, 0), (2, 30, 11, 5),
            (1, 0, 0, 64), (2, 0, 0, 64)]


@pytest.mark.parametrize("n,with_f,iters", [
    (1, True, 5), (2, False, 7), (3, True, 9), (5, True, 11), (16, False, 13),
    (33, True, 17), (64, True, 6), (67, False, 9), (130, True, 4)])
def test_fixed_iterations_bitwise(sor, ctx, n, with_f, iters):
    g = random_cube(300 + n, n, with_f=with_f, nonzero_u0=True)
    ref = oracle.sor3d_f64(g.u0, g.bdy, g.f, g.omega, 0.0, iters, 1, threads=8, hist=True)
    for T, cx, cy, zs in TILINGS3:
        K = 2 if T != 1 else 1        # tol 0: the check cadence changes nothing else
        _say(f"3d stream n={n} f={with_f} iters={iters} T={T} tiling=({cx},{cy},{zs})")
        ctx.set_tiling3d(cx, cy, zs, iters=T)
        res, u = run3(sor, ctx, g, 0.0, iters, K)
        assert res.status == sor.NOT_CONVERGED and res.iterations == iters
        assert_bitwise(u, ref.u, f"u n={n} T={T} tiling=({cx},{cy},{zs})")
        assert_bitwise(np.array(res.hist), ref.mhist, f"hist n={n} T={T} tiling=({cx},{cy},{zs})")
    _say(f"3d colour kernel n={n}")
    ctx.set_tiling3d(0, 0, 0)
    ctx.set_kernel(sor.KERNEL_SIMPLE)
    res, u = run3(sor, ctx, g, 0.0, iters, 1)
    assert_bitwise(u, ref.u, f"u n={n} colour kernel")
    assert_bitwise(np.array(res.hist), ref.mhist, f"hist n={n} colour kernel")


@pytest.mark.parametrize("omega", [0.376, 1.0, 1.5, 1.95])
def test_omega_values_bitwise(sor, ctx, omega):
    g = random_cube(77, 21, with_f=True, omega=omega)
    _say(f"3d omega={omega}")
    ref = oracle.sor3d_f64(g.u0, g.bdy, g.f, omega, 0.0, 25, 1, threads=8, hist=True)
    res, u = run3(sor, ctx, g, 0.0, 25, 1)
    assert_bitwise(u, ref.u, f"u omega={omega}")
    assert_bitwise(np.array(res.hist), ref.mhist, f"hist omega={omega}")


@pytest.mark.parametrize("K", [1, 2, 5, 10])
def test_to_tolerance_same_stop(sor, ctx, K):
    """Converges; stops at the same checked iteration with the same change
    and the same grid (the chunked host loop never overshoots the stop, and
    the result is taken from whichever grid the last executed pass wrote:
    tolerances met at odd and at even iterations)."""
    n = 24
    g = random_cube(11, n, with_f=False)
    for tol in (1e-3, 1e-5, 1e-8):
        _say(f"3d tol={tol} K={K}")
        ref = oracle.sor3d_f64(g.u0, g.bdy, None, g.omega, tol, 100000, K, threads=8, hist=True)
        assert ref.status == oracle.OK
        res, u = run3(sor, ctx, g, tol, 100000, K)
        assert res.status == sor.OK and res.converged
        assert res.iterations == ref.iterations and res.iterations % K == 0
        assert res.final_max_delta == ref.final_max_delta
        assert_bitwise(u, ref.u, "u")
        assert_bitwise(np.array(res.hist), ref.mhist, "hist")


def test_poisson_to_tolerance_and_max_iters_check(sor, ctx):
    """A solve that ends at max_iters (not a multiple of K) checks there."""
    n = 31
    g = random_cube(12, n, with_f=True)
    ref = oracle.sor3d_f64(g.u0, g.bdy, g.f, g.omega, 1e-12, 173, 10, threads=8)
    res, u = run3(sor, ctx, g, 1e-12, 173, 10, hist=False)
    assert res.status == sor.NOT_CONVERGED and ref.status == oracle.NOT_CONVERGED
    assert res.iterations == 173 and res.final_max_delta == ref.final_max_delta
    assert_bitwise(u, ref.u, "u")


def test_sampled_cells_at_256_against_converged_oracle(sor, ctx):
    """n = 256 at the bench's configuration: run the same fixed iteration count
    on both sides and compare the full grid (the oracle at 8 threads)."""
    n = 256
    g = random_cube(9, n, with_f=False)
    iters = 21
    _say("3d n=256 oracle")
    ref = oracle.sor3d_f64(g.u0, g.bdy, None, g.omega, 0.0, iters, 1, threads=8, hist=True)
    for K in (1, 10):                 # one, then two iterations per launch
        _say(f"3d n=256 gpu K={K}")
        res, u = run3(sor, ctx, g, 0.0, iters, K)
        assert_bitwise(u, ref.u, f"u n=256 K={K}")
        assert_bitwise(np.array(res.hist), ref.mhist, f"hist n=256 K={K}")


def test_tiling3d_reporting_and_rejection(sor, ctx):
    T, cx, cy, zs = ctx.tiling3d_for(256)
    assert T == 1 and (cx + 4) * (cy + 4) <= 2048 and 1 <= zs <= 256
    T, cx, cy, zs = ctx.tiling3d_for(256, check_every=10)
    assert T == 2 and (cx + 8) * (cy + 8) <= 2032 and 1 <= zs <= 256
    assert ctx.tiling3d_for(256, has_rhs=True, check_every=10)[0] == 2   # with a source too
    ctx.set_tiling3d(30, 11, 5)
    assert ctx.tiling3d_for(256) == (1, 29, 11, 5)     # 9 equal strips of <= 30
    assert ctx.tiling3d_for(256, check_every=4) == (2, 29, 11, 5)
    ctx.set_tiling3d(30, 11, 5, iters=1)
    assert ctx.tiling3d_for(256, check_every=4) == (1, 29, 11, 5)
    for bad in ((-1, 0, 0, 0), (0, -2, 0, 0), (0, 0, -3, 0), (500, 0, 0, 0), (60, 60, 0, 0),
                (0, 0, 0, 3), (0, 0, 0, -1), (40, 40, 0, 2)):
        with pytest.raises(sor.SorError):
            ctx.set_tiling3d(*bad[:3], iters=bad[3])
    ctx.set_tiling3d(0, 0, 0)


@pytest.mark.parametrize("n,scale,first_bad", [(41, 0.12, 3), (20, 0.15, 2)])
def test_overflow_during_solve_reported(sor, ctx, n, scale, first_bad):
    """Finite faces at a fraction of the largest double: over-relaxation
    overshoots and a neighbour sum overflows a few iterations in, between two
    checks (K = 10).  Every launch shape stops with ENONFINITE by the end of
    the launch holding the oracle's first infinite change, with the same
    changes up to and including it."""
    from workloads import Grid
    top = float(np.finfo(np.float64).max)
    g = Grid(n, np.zeros((n, n, n)), np.full((6, n, n), scale * top), None, omega_opt(n))
    ref = oracle.sor3d_f64(g.u0, g.bdy, None, g.omega, 0.0, 100, 10, hist=True)
    assert ref.status == oracle.ENONFINITE and ref.iterations == first_bad
    for t in [(0, 0, 0, 0), (1, 0, 0, 0), (2, 0, 0, 0), (2, 4, 3, 3), (1, 7, 5, 1)]:
        _say(f"overflow 3d n={n} scale={scale} tiling={t}")
        ctx.set_tiling3d(*t[1:], iters=t[0])
        res, _ = run3(sor, ctx, g, 0.0, 100, 10)
        assert res.status == sor.ENONFINITE and not res.converged, (t, res)
        assert first_bad <= res.iterations < first_bad + 2, (t, res.iterations)
        assert_bitwise(res.hist[:first_bad], ref.mhist, f"changes up to the overflow, {t}")
    ctx.set_tiling3d(0, 0, 0)
    _say(f"overflow 3d n={n} scale={scale} colour kernel")
    ctx.set_kernel(sor.KERNEL_SIMPLE)
    res, _ = run3(sor, ctx, g, 0.0, 100, 10)
    ctx.set_kernel(sor.KERNEL_BLOCKED)
    assert res.status == sor.ENONFINITE and res.iterations == first_bad, res
    assert_bitwise(res.hist[:first_bad], ref.mhist, "changes up to the overflow, colour kernel")


def test_nonfinite_input_and_invalid_arguments(sor, ctx):
    n = 9
    g = random_cube(5, n, with_f=True)
    bdy = g.bdy.copy()
    bdy[3, 4, 4] = np.inf
    ref = oracle.sor3d_f64(g.u0, bdy, g.f, g.omega, 1e-8, 50, 1)
    assert ref.status == oracle.ENONFINITE
    res = sor.solve3d_f64(dev(g.u0), dev(bdy), dev(g.f), g.omega, 1e-8, 50, 1, ctx=ctx)
    assert res.status == sor.ENONFINITE and not res.converged
    with pytest.raises(sor.SorError):
        sor.solve3d_f64(dev(g.u0), dev(g.bdy), None, 2.0, 1e-8, 10, 1, ctx=ctx)
    with pytest.raises(sor.SorError):
        sor.solve3d_f64(dev(g.u0), dev(g.bdy), None, 1.5, 1e-8, 0, 1, ctx=ctx)
    # the context stays usable after the errors
    ref = oracle.sor3d_f64(g.u0, g.bdy, g.f, g.omega, 0.0, 8, 1, hist=True)
    res, u = run3(sor, ctx, g, 0.0, 8, 1)
    assert_bitwise(u, ref.u, "u after errors")
