"""The allocation-free FP64 solve (sor_solve_f64_noalloc) against sor_solve_f64.

Both are called through the C ABI on the same seeded inputs; the allocation-
free call must give the same u, result and per-iteration changes bit for bit.
Consecutive calls share the library's fixed working region, so the checks run
two calls in a row, the second on a smaller grid than the first, plus a
Laplace call after a Poisson one (the second must not read the first's
source).  Sizes beyond the region are rejected before any device work.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1401_0763_amd as sor  # noqa: E402
from workloads import random_small  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda:0")


def _pair(ctx, g, tol, iters, K, with_f):
    """Run the grid through both entry points; return both (u, result)."""
    out = []
    for fn in (sor.solve_f64, sor.solve_f64_noalloc):
        u = _dev(g.u0)
        res = fn(u, _dev(g.bdy), _dev(g.f) if with_f else None, g.omega, tol, iters,
                 K, hist=True, ctx=ctx)
        out.append((u.cpu().numpy(), res))
    return out


def _same(a, b):
    (ua, ra), (ub, rb) = a, b
    assert np.array_equal(ua.view(np.uint64), ub.view(np.uint64)), \
        f"max diff {np.abs(ua - ub).max()}"
    assert (ra.status, ra.iterations, ra.converged) == (rb.status, rb.iterations, rb.converged)
    assert np.array_equal(np.array([ra.final_max_delta]).view(np.uint64),
                          np.array([rb.final_max_delta]).view(np.uint64))
    assert np.array_equal(np.array(ra.hist), np.array(rb.hist))


@pytest.mark.parametrize("first,second", [(700, 130), (1583, 257)])
def test_two_calls_in_a_row_second_smaller(first, second):
    ctx = sor.Context(0)
    try:
        # First: Poisson with a nonzero start, fixed count ending inside a pass.
        g1 = random_small(31, first, with_f=True, nonzero_u0=True)
        a, b = _pair(ctx, g1, 0.0, 45, 1, True)
        _same(a, b)
        assert b[1].iterations == 45 and b[1].status == sor.NOT_CONVERGED
        # Second: smaller Laplace grid solved to a tolerance (the stop falls
        # inside a pass and is re-run from the pass input).
        g2 = random_small(32, second, with_f=False, nonzero_u0=False)
        a, b = _pair(ctx, g2, 1e-6, 20000, 1, False)
        _same(a, b)
        assert b[1].status == sor.OK and b[1].converged
    finally:
        ctx.close()


def test_largest_laplace_grid_and_check_cadence():
    ctx = sor.Context(0)
    try:
        g = random_small(33, 1951, with_f=False, nonzero_u0=True)
        a, b = _pair(ctx, g, 0.0, 23, 10, False)
        _same(a, b)
        g = random_small(34, 64, with_f=True, nonzero_u0=False)
        a, b = _pair(ctx, g, 1e-9, 5000, 7, True)
        _same(a, b)
        assert b[1].iterations % 7 == 0 or b[1].iterations == 5000
    finally:
        ctx.close()


def test_sizes_beyond_the_region_are_rejected():
    ctx = sor.Context(0)
    try:
        for n, with_f in ((1952, False), (1584, True)):
            u = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
            bdy = torch.ones(4 * n, dtype=torch.float64, device="cuda:0")
            f = torch.zeros((n, n), dtype=torch.float64, device="cuda:0") if with_f else None
            with pytest.raises(sor.SorError) as e:
                sor.solve_f64_noalloc(u, bdy, f, 1.5, 0.0, 3, 1, ctx=ctx)
            assert e.value.status == sor.EINVAL
            assert "n <= 1951 without a source" in str(e.value)
            assert "n <= 1583 with one" in str(e.value)
            assert float(u.abs().max()) == 0.0        # no device work was done
        # The region is still usable after a rejection.
        g = random_small(35, 96, with_f=True, nonzero_u0=True)
        a, b = _pair(ctx, g, 0.0, 17, 1, True)
        _same(a, b)
    finally:
        ctx.close()


def test_simple_kernel_and_nonfinite_input():
    ctx = sor.Context(0)
    try:
        ctx.set_kernel(sor.KERNEL_SIMPLE)
        g = random_small(36, 200, with_f=True, nonzero_u0=True)
        a, b = _pair(ctx, g, 0.0, 9, 1, True)
        _same(a, b)
        ctx.set_kernel(sor.KERNEL_BLOCKED)
        g = random_small(37, 150, with_f=False, nonzero_u0=True)
        g.u0[40, 77] = np.inf
        a, b = _pair(ctx, g, 0.0, 12, 1, False)
        assert a[1].status == sor.ENONFINITE and b[1].status == sor.ENONFINITE
        assert a[1].iterations == b[1].iterations
        # A clean solve after the non-finite one is unaffected by what it left.
        g = random_small(38, 150, with_f=False, nonzero_u0=True)
        a, b = _pair(ctx, g, 0.0, 12, 1, False)
        _same(a, b)
    finally:
        ctx.close()
