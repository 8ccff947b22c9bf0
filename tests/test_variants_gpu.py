"""GPU parity of the Jacobi and four-colour orderings (the alternatives to
red-black named in Sec. 2.1 and Sec. 3.1 of Mittal 2014) against the oracle
on identical seeded inputs: final grid, every iteration's largest change and
the stop iteration agree bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from workloads import laplace_random_boundary, random_small

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


ORDERS = [(1, "jacobi"), (2, "four-colour")]


def run(sor, ctx, ordering, g, omega, tol, iters, K, hist=True):
    u = dev(g.u0)
    res = sor.solve_variant_f64(ordering, u, dev(g.bdy), dev(g.f), omega, tol, iters, K,
                                hist=hist, ctx=ctx)
    return res, u.cpu().numpy()


@pytest.mark.parametrize("ordering,name", ORDERS)
@pytest.mark.parametrize("n,with_f,iters", [
    (1, True, 5), (2, False, 6), (3, True, 7), (17, True, 11), (64, False, 9),
    (100, True, 13), (255, True, 8), (513, False, 6), (600, True, 5)])
def test_fixed_iterations_bitwise(sor, ctx, ordering, name, n, with_f, iters):
    g = random_small(700 + n, n, with_f=with_f, nonzero_u0=True)
    for omega in (1.0, 1.37):
        _say(f"{name} n={n} f={with_f} iters={iters} omega={omega}")
        ref = oracle.variant_f64(ordering, g.u0, g.bdy, g.f, omega, 0.0, iters, 1, hist=True)
        res, u = run(sor, ctx, ordering, g, omega, 0.0, iters, 1)
        assert res.status == sor.NOT_CONVERGED and res.iterations == iters
        assert_bitwise(u, ref.u, f"{name} u n={n}")
        assert_bitwise(np.array(res.hist), ref.mhist, f"{name} hist n={n}")


@pytest.mark.parametrize("ordering,name", ORDERS)
@pytest.mark.parametrize("K", [1, 4, 10])
def test_to_tolerance_same_stop(sor, ctx, ordering, name, K):
    """Stops at the same checked iteration (odd and even, so the Jacobi
    result is read from either grid) with the same change and grid."""
    n = 40
    g = random_small(41, n, with_f=True)
    omega = 1.0 if ordering == 1 else g.omega
    for tol in (1e-2, 1e-5, 1e-9):
        ref = oracle.variant_f64(ordering, g.u0, g.bdy, g.f, omega, tol, 50000, K, hist=True)
        _say(f"{name} K={K} tol={tol} ref_it={ref.iterations}")
        assert ref.status == oracle.OK
        res, u = run(sor, ctx, ordering, g, omega, tol, 50000, K)
        assert res.status == sor.OK and res.converged
        assert res.iterations == ref.iterations
        assert res.final_max_delta == ref.final_max_delta
        assert_bitwise(u, ref.u, f"{name} u tol={tol}")
        assert_bitwise(np.array(res.hist), ref.mhist, f"{name} hist tol={tol}")


@pytest.mark.parametrize("ordering,name", ORDERS)
def test_max_iters_not_multiple_of_k(sor, ctx, ordering, name):
    n = 33
    g = random_small(5, n, with_f=False)
    ref = oracle.variant_f64(ordering, g.u0, g.bdy, None, 1.2, 1e-14, 57, 10)
    res, u = run(sor, ctx, ordering, g, 1.2, 1e-14, 57, 10, hist=False)
    assert res.status == sor.NOT_CONVERGED and ref.status == oracle.NOT_CONVERGED
    assert res.iterations == 57 and res.final_max_delta == ref.final_max_delta
    assert_bitwise(u, ref.u, f"{name} u")


@pytest.mark.parametrize("ordering,name", ORDERS)
def test_bench_grid_4096(sor, ctx, ordering, name):
    """The 4096^2 bench grid, 4 iterations, whole grid compared."""
    g = laplace_random_boundary(4096)
    omega = 1.0 if ordering == 1 else g.omega
    _say(f"{name} 4096 oracle")
    ref = oracle.variant_f64(ordering, g.u0, g.bdy, None, omega, 0.0, 4, 1, hist=True)
    _say(f"{name} 4096 gpu")
    res, u = run(sor, ctx, ordering, g, omega, 0.0, 4, 1)
    assert_bitwise(u, ref.u, f"{name} u 4096")
    assert_bitwise(np.array(res.hist), ref.mhist, f"{name} hist 4096")


def test_red_black_ordering_is_solve_f64_and_errors(sor, ctx):
    n = 20
    g = random_small(9, n, with_f=True)
    ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 0.0, 12, 1)
    res, u = run(sor, ctx, 0, g, g.omega, 0.0, 12, 1, hist=False)
    assert_bitwise(u, ref.u, "red-black via the ordering entry point")
    with pytest.raises(sor.SorError):
        run(sor, ctx, 3, g, 1.0, 0.0, 5, 1)
    with pytest.raises(sor.SorError):
        run(sor, ctx, 1, g, 2.0, 0.0, 5, 1)
    bdy = g.bdy.copy()
    bdy[7] = np.nan
    for ordering, name in ORDERS:
        assert oracle.variant_f64(ordering, g.u0, bdy, g.f, 1.0, 1e-6, 50, 1).status == oracle.ENONFINITE
        u = dev(g.u0)
        r = sor.solve_variant_f64(ordering, u, dev(bdy), dev(g.f), 1.0, 1e-6, 50, 1, ctx=ctx)
        assert r.status == sor.ENONFINITE, name


@pytest.mark.parametrize("ordering,n,scale,first_bad", [
    (1, 37, 0.3, 7), (1, 130, 0.35, 3), (2, 130, 0.15, 7), (2, 37, 0.25, 2)])
def test_overflow_during_solve_reported(sor, ctx, ordering, n, scale, first_bad):
    """Finite inputs whose iterates overflow between two checks (K = 10): a
    uniform boundary at a fraction of the largest double.  Blocked passes of
    several depths and the one-iteration kernel stop with ENONFINITE by the
    end of the pass holding the oracle's first infinite change, with the same
    changes up to and including it."""
    from workloads import Grid, omega_opt
    top = float(np.finfo(np.float64).max)
    omega = 1.0 if ordering == 1 else omega_opt(n)
    g = Grid(n, np.zeros((n, n)), np.full(4 * n, scale * top), None, omega)
    ref = oracle.variant_f64(ordering, g.u0, g.bdy, None, omega, 0.0, 100, 10, hist=True)
    assert ref.status == oracle.ENONFINITE and ref.iterations == first_bad
    depths = (1, 3, 8) if ordering == 1 else (1, 3, 5)
    for T in depths + (0,):
        _say(f"overflow ordering={ordering} n={n} scale={scale} T={T}")
        if T:
            ctx.set_kernel(sor.KERNEL_BLOCKED)
            ctx.set_variant_tiling(ordering, T, 0)
        else:
            ctx.set_kernel(sor.KERNEL_SIMPLE)
        res, _ = run(sor, ctx, ordering, g, omega, 0.0, 100, 10)
        assert res.status == sor.ENONFINITE and not res.converged, (T, res)
        assert first_bad <= res.iterations < first_bad + max(T, 1), (T, res.iterations)
        assert_bitwise(res.hist[:first_bad], ref.mhist, f"changes up to the overflow, T={T}")


# Blocked passes of both orderings: every depth (truncated passes when fewer
# iterations remain), segment heights that do and do not divide the grid, and
# strips with a ragged last one.
BLOCKED_TILINGS = [
    (2, "four-colour", 1, 8), (2, "four-colour", 2, 14), (2, "four-colour", 3, 30),
    (2, "four-colour", 4, 48), (2, "four-colour", 4, 202), (2, "four-colour", 3, 64),
    (2, "four-colour", 2, 1024), (2, "four-colour", 5, 40), (2, "four-colour", 5, 110),
    (1, "jacobi", 1, 8), (1, "jacobi", 2, 14), (1, "jacobi", 3, 30), (1, "jacobi", 4, 48),
    (1, "jacobi", 5, 40), (1, "jacobi", 6, 202), (1, "jacobi", 7, 64), (1, "jacobi", 8, 16),
    (1, "jacobi", 8, 1024)]


@pytest.mark.parametrize("ordering,name,T,seg", BLOCKED_TILINGS)
@pytest.mark.parametrize("n,with_f,iters", [
    (1, False, 3), (5, True, 9), (61, True, 11), (130, False, 13), (300, True, 10),
    (513, False, 7)])
def test_blocked_tilings_bitwise(sor, ctx, ordering, name, T, seg, n, with_f, iters):
    g = random_small(900 + n + T, n, with_f=with_f, nonzero_u0=True)
    ctx.set_variant_tiling(ordering, T, seg)
    assert ctx.get_variant_tiling(ordering) == (T, seg)
    _say(f"{name} blocked T={T} seg={seg} n={n} f={with_f} iters={iters}")
    ref = oracle.variant_f64(ordering, g.u0, g.bdy, g.f, 1.37, 0.0, iters, 1, hist=True)
    res, u = run(sor, ctx, ordering, g, 1.37, 0.0, iters, 1)
    assert res.status == sor.NOT_CONVERGED and res.iterations == iters
    assert res.passes == -(-iters // T)     # every pass did work (no early stop)
    assert_bitwise(u, ref.u, f"{name} blocked u T={T} seg={seg} n={n}")
    assert_bitwise(np.array(res.hist), ref.mhist, f"{name} blocked hist T={T} n={n}")


@pytest.mark.parametrize("ordering,name,T", [
    (2, "four-colour", 2), (2, "four-colour", 3), (2, "four-colour", 4), (2, "four-colour", 5),
    (1, "jacobi", 3), (1, "jacobi", 8)])
@pytest.mark.parametrize("K", [1, 3, 5])
def test_blocked_stop_inside_a_pass(sor, ctx, ordering, name, T, K):
    """Checks that fall inside a pass: the pass is redone up to the stop from
    its intact input, so grid and change match the oracle's stop."""
    n = 90
    g = random_small(77 + K, n, with_f=True)
    omega = 1.0 if ordering == 1 else g.omega
    ctx.set_variant_tiling(ordering, T, 32)
    for tol in ((1e-2, 1e-4) if ordering == 1 else (1e-3, 1e-7)):
        ref = oracle.variant_f64(ordering, g.u0, g.bdy, g.f, omega, tol, 50000, K, hist=True)
        _say(f"{name} blocked T={T} K={K} tol={tol} ref_it={ref.iterations}")
        assert ref.status == oracle.OK
        res, u = run(sor, ctx, ordering, g, omega, tol, 50000, K)
        assert res.status == sor.OK and res.iterations == ref.iterations
        assert res.final_max_delta == ref.final_max_delta
        assert_bitwise(u, ref.u, f"{name} blocked u T={T} K={K} tol={tol}")
        assert_bitwise(np.array(res.hist), ref.mhist, f"{name} blocked hist T={T} K={K}")


@pytest.mark.parametrize("ordering,name,default_T", [(2, "four-colour", 5), (1, "jacobi", 8)])
def test_simple_and_blocked_agree(sor, ctx, ordering, name, default_T):
    """The one-iteration-per-launch kernels and the blocked passes give the
    same bits (and the oracle's)."""
    n = 257
    g = random_small(31, n, with_f=True, nonzero_u0=True)
    ref = oracle.variant_f64(ordering, g.u0, g.bdy, g.f, g.omega, 0.0, 14, 1, hist=True)
    ctx.set_kernel(sor.KERNEL_SIMPLE)
    res_s, u_s = run(sor, ctx, ordering, g, g.omega, 0.0, 14, 1)
    assert res_s.passes == 14
    ctx.set_kernel(sor.KERNEL_BLOCKED)
    res_b, u_b = run(sor, ctx, ordering, g, g.omega, 0.0, 14, 1)
    assert res_b.passes == -(-14 // default_T)
    assert_bitwise(u_s, ref.u, f"{name} simple")
    assert_bitwise(u_b, ref.u, f"{name} blocked")
    assert_bitwise(np.array(res_s.hist), ref.mhist, f"{name} simple hist")
    assert_bitwise(np.array(res_b.hist), ref.mhist, f"{name} blocked hist")


def test_variant_tiling_validation(sor, ctx):
    assert ctx.get_variant_tiling(sor.ORDER_FOUR_COLOUR) == (5, 0)
    assert ctx.get_variant_tiling(sor.ORDER_JACOBI) == (8, 0)
    for ordering, bad in [(sor.ORDER_FOUR_COLOUR, (6, 0)), (sor.ORDER_JACOBI, (9, 0))]:
        with pytest.raises(sor.SorError):
            ctx.set_variant_tiling(ordering, *bad)
    for bad in [(0, 7), (0, 6), (0, 1026), (-1, 0)]:
        for ordering in (sor.ORDER_FOUR_COLOUR, sor.ORDER_JACOBI):
            with pytest.raises(sor.SorError):
                ctx.set_variant_tiling(ordering, *bad)
    for ordering in (sor.ORDER_RED_BLACK, 7):
        with pytest.raises(sor.SorError):
            ctx.set_variant_tiling(ordering, 2, 64)
    ctx.set_variant_tiling(sor.ORDER_FOUR_COLOUR, 0, 96)
    assert ctx.get_variant_tiling(sor.ORDER_FOUR_COLOUR) == (5, 96)
    ctx.set_variant_tiling(sor.ORDER_JACOBI, 5, 0)
    assert ctx.get_variant_tiling(sor.ORDER_JACOBI) == (5, 0)
