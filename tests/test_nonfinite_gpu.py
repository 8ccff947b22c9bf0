"""GPU handling of values that turn non-finite from finite operands.

A NaN can come straight out of finite data: (+inf) + (-inf) when one
neighbour pair overflows upwards and the other downwards.  Its change |new -
old| is NaN, which a running maximum drops, so the stopping rule alone would
read such an iteration as converged.  The oracle checks every update; the
GPU passes check every interior cell they store (non-finite values are
absorbing for interior cells, so a cell that went non-finite anywhere in a
pass is non-finite at its end).  When the stopping rule is met at an
iteration inside a pass that also made a non-finite value, the truncated
re-run of that pass decides which came first.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import Grid, omega_opt

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


def big(bits):
    return float(np.finfo(np.float64 if bits == 64 else np.float32).max)


def opposite_boundary(n, bits):
    """North and south at +0.6 max, west and east at -0.6 max: for n = 1 the
    one cell's neighbour sum is (+inf) + (-inf) = NaN at iteration 1."""
    v = 0.6 * big(bits)
    if bits == 32:
        v = float(np.float32(v))
    return Grid(n, np.zeros((n, n)), np.concatenate([np.full(2 * n, v), np.full(2 * n, -v)]),
                None, omega_opt(n))


def interior_cross(n, bits):
    """Zero boundary (1.0), and around the interior cell (65, 65) (red) the
    initial values +0.6 max north and south, -0.6 max west and east: that
    cell's sum is NaN in the first red phase while every change of the
    iteration stays finite."""
    v = 0.6 * big(bits)
    if bits == 32:
        v = float(np.float32(v))
    u0 = np.zeros((n, n))
    c = 64
    u0[c - 1, c] = u0[c + 1, c] = v
    u0[c, c - 1] = u0[c, c + 1] = -v
    return Grid(n, u0, np.full(4 * n, 1.0), None, omega_opt(n))


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def solve(sor, ctx, g, bits, tol, iters, K, ordering=0):
    dtype = torch.float64 if bits == 64 else torch.float32
    u = dev(g.u0, dtype)
    if ordering:
        res = sor.solve_variant_f64(ordering, u, dev(g.bdy, dtype), None, g.omega, tol, iters,
                                    K, hist=True, ctx=ctx)
    else:
        fn = sor.solve_f64 if bits == 64 else sor.solve_f32
        res = fn(u, dev(g.bdy, dtype), None, g.omega, tol, iters, K, hist=True, ctx=ctx)
    return res, u.cpu().numpy()


def reference(g, bits, tol, iters, K, ordering=0):
    if ordering:
        return oracle.variant_f64({1: oracle.ORDER_JACOBI, 2: oracle.ORDER_FOUR_COLOUR}[ordering],
                                  g.u0, g.bdy, None, g.omega, tol, iters, K, hist=True)
    if bits == 64:
        return oracle.sor_f64(g.u0, g.bdy, None, g.omega, tol, iters, K, hist=True)
    return oracle.sor_f32(g.u0.astype(np.float32), g.bdy.astype(np.float32), None, g.omega,
                          tol, iters, K, hist=True)


TILINGS = [(1, 8), (2, 16), (4, 64), (7, 94), (8, 16), (0, 0)]


@pytest.mark.parametrize("make", [opposite_boundary, interior_cross])
@pytest.mark.parametrize("bits", [64, 32])
def test_nan_from_finite_operands_reported(sor, ctx, make, bits):
    n = 1 if make is opposite_boundary else 130
    g = make(n, bits)
    ref = reference(g, bits, 0.0, 30, 10)
    assert ref.status == oracle.ENONFINITE and ref.iterations == 1
    assert np.isfinite(ref.mhist).all()              # the maxima never show it
    for T, seg in TILINGS:
        _say(f"nan-from-finite {make.__name__} bits={bits} n={n} T={T} seg={seg}")
        if T:
            ctx.set_kernel(sor.KERNEL_BLOCKED)
            ctx.set_tiling(bits, T, seg)
        else:
            ctx.set_kernel(sor.KERNEL_SIMPLE)
        res, _ = solve(sor, ctx, g, bits, 0.0, 30, 10)
        assert res.status == sor.ENONFINITE and not res.converged, (T, res)
        assert 1 <= res.iterations <= max(T, 1), (T, res.iterations)


@pytest.mark.parametrize("ordering", [1, 2])
@pytest.mark.parametrize("make", [opposite_boundary, interior_cross])
def test_nan_from_finite_operands_orderings(sor, ctx, make, ordering):
    n = 1 if make is opposite_boundary else 130
    g = make(n, 64)
    g.omega = 1.0 if ordering == 1 else g.omega
    ref = reference(g, 64, 0.0, 30, 10, ordering)
    assert ref.status == oracle.ENONFINITE, ref.status
    for kernel in (sor.KERNEL_BLOCKED, sor.KERNEL_SIMPLE):
        _say(f"nan-from-finite ordering={ordering} {make.__name__} kernel={kernel}")
        ctx.set_kernel(kernel)
        res, _ = solve(sor, ctx, g, 64, 0.0, 30, 10, ordering)
        assert res.status == sor.ENONFINITE, (kernel, res)
        assert ref.iterations <= res.iterations <= ref.iterations + 8, (kernel, res.iterations)


def test_nan_from_finite_operands_in_a_batch(sor, ctx):
    grids = [interior_cross(130, 64), opposite_boundary(1, 64)]
    rng = np.random.default_rng(3)
    ok = Grid(70, np.zeros((70, 70)), rng.uniform(0, 100, 280), None, omega_opt(70))
    grids.append(ok)
    specs, us = [], []
    for g in grids:
        u = dev(g.u0, torch.float64)
        us.append(u)
        specs.append(sor.GridSpec(u, dev(g.bdy, torch.float64), None, g.omega, 0.0, 30, 10))
    _say("nan-from-finite batch")
    res = sor.batch_solve_f64(specs, ctx=ctx)
    assert res[0].status == sor.ENONFINITE and res[1].status == sor.ENONFINITE
    assert res[2].status == sor.NOT_CONVERGED
    ref = oracle.sor_f64(ok.u0, ok.bdy, None, ok.omega, 0.0, 30, 10)
    got = us[2].cpu().numpy()
    assert np.array_equal(got.view(np.uint64), ref.u.view(np.uint64))


@pytest.mark.parametrize("bits", [64, 32])
def test_stop_inside_pass_before_overflow_converges(sor, ctx, bits):
    """With tol = inf and a check every iteration the rule passes at iteration
    1; the iterates of a boundary at 0.15 of the largest finite value overflow
    at iteration 6, inside the same pass.  The oracle stops at iteration 1
    with a finite grid, and so must every tiling."""
    n = 130
    v = 0.15 * big(bits)
    if bits == 32:
        v = float(np.float32(v))
    g = Grid(n, np.zeros((n, n)), np.full(4 * n, v), None, omega_opt(n))
    ref = reference(g, bits, float("inf"), 100, 1)
    assert ref.status == oracle.OK and ref.iterations == 1
    assert reference(g, bits, 0.0, 100, 10).iterations == 6       # the overflow
    for T, seg in TILINGS:
        _say(f"tentative stop bits={bits} T={T}")
        if T:
            ctx.set_kernel(sor.KERNEL_BLOCKED)
            ctx.set_tiling(bits, T, seg)
        else:
            ctx.set_kernel(sor.KERNEL_SIMPLE)
        res, u = solve(sor, ctx, g, bits, float("inf"), 100, 1)
        assert res.status == sor.OK and res.iterations == 1, (T, res)
        view = np.uint64 if bits == 64 else np.uint32
        assert np.array_equal(u.view(view), ref.u.view(view)), T


@pytest.mark.parametrize("bits", [64, 32])
def test_stop_inside_pass_after_nan_is_nonfinite(sor, ctx, bits):
    """tol = inf, checked every iteration: the n = 1 opposite boundary makes a
    NaN at iteration 1 whose change (NaN) the maximum drops, so the rule also
    'passes' at iteration 1.  The oracle reports the non-finite value; the
    truncated re-run must find it too."""
    g = opposite_boundary(1, bits)
    ref = reference(g, bits, float("inf"), 100, 1)
    assert ref.status == oracle.ENONFINITE and ref.iterations == 1
    for T, seg in TILINGS:
        _say(f"tentative nan bits={bits} T={T}")
        if T:
            ctx.set_kernel(sor.KERNEL_BLOCKED)
            ctx.set_tiling(bits, T, seg)
        else:
            ctx.set_kernel(sor.KERNEL_SIMPLE)
        res, _ = solve(sor, ctx, g, bits, float("inf"), 100, 1)
        assert res.status == sor.ENONFINITE, (T, res)
        assert res.iterations == 1, (T, res.iterations)
