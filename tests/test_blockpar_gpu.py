"""GPU parity of block-parallel SOR (the parallel SOR form that Sec. 3.1 of
Mittal 2014 names; blocks updated together, red-black inside a block, a
neighbour in another block at the previous iterate) against the oracle on
identical seeded inputs: final grid, every iteration's largest change and the
stop iteration agree bit for bit, for every pass depth, tilings whose tiles
cut blocks anywhere, ragged blocks and grids, and the two limits.  Blocks of
even width (or wider than the grid) run a kernel of their own, so the cases
mix even and odd widths."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Grid, laplace_random_boundary, random_small

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


def run(sor, ctx, g, br, bc, omega, tol, iters, K, hist=True):
    u = dev(g.u0)
    res = sor.solve_blockpar_f64(u, dev(g.bdy), br, bc, dev(g.f), omega, tol, iters, K,
                                 hist=hist, ctx=ctx)
    return res, u.cpu().numpy()


def check(sor, ctx, g, br, bc, omega, iters, what):
    ref = oracle.blockpar_f64(g.u0, g.bdy, g.f, omega, br, bc, 0.0, iters, 1, hist=True)
    res, u = run(sor, ctx, g, br, bc, omega, 0.0, iters, 1)
    assert res.status == sor.NOT_CONVERGED and res.iterations == iters, (what, res)
    assert_bitwise(u, ref.u, f"{what} u")
    assert_bitwise(np.array(res.hist), ref.mhist, f"{what} hist")
    return res


SHAPES = [(1, 1), (2, 2), (3, 5), (16, 16), (64, 7), (1, 1000), (1000, 3), (4096, 4096)]


@pytest.mark.parametrize("br,bc", SHAPES)
@pytest.mark.parametrize("n,with_f,iters", [
    (1, True, 5), (2, False, 6), (3, True, 7), (17, True, 11), (64, False, 9),
    (100, True, 13), (255, True, 8), (513, False, 6), (600, True, 5)])
def test_fixed_iterations_bitwise(sor, ctx, br, bc, n, with_f, iters):
    g = random_small(1300 + n, n, with_f=with_f, nonzero_u0=True)
    for omega in (1.0, 1.25):
        _say(f"blockpar {br}x{bc} n={n} f={with_f} iters={iters} omega={omega}")
        check(sor, ctx, g, br, bc, omega, iters, f"{br}x{bc} n={n} omega={omega}")


# Every depth, segment heights that do and do not divide the grid, and block
# widths that do and do not line up with the strips (core width 128 - 4T).
BLOCKED_TILINGS = [(1, 8), (2, 14), (3, 30), (4, 48), (5, 40), (5, 202), (6, 64), (7, 94),
                   (8, 16), (8, 1024)]


@pytest.mark.parametrize("T,seg", BLOCKED_TILINGS)
@pytest.mark.parametrize("n,with_f,iters,br,bc", [
    (1, False, 3, 1, 1), (5, True, 9, 2, 3), (61, True, 11, 7, 9), (130, False, 13, 30, 108),
    (300, True, 10, 13, 50), (513, False, 7, 64, 64)])
def test_blocked_tilings_bitwise(sor, ctx, T, seg, n, with_f, iters, br, bc):
    g = random_small(1900 + n + T, n, with_f=with_f, nonzero_u0=True)
    ctx.set_variant_tiling(sor.ORDER_BLOCK_PARALLEL, T, seg)
    assert ctx.get_variant_tiling(sor.ORDER_BLOCK_PARALLEL) == (T, seg)
    _say(f"blockpar T={T} seg={seg} n={n} blocks {br}x{bc} iters={iters}")
    res = check(sor, ctx, g, br, bc, 1.2, iters, f"T={T} seg={seg} n={n} {br}x{bc}")
    assert res.passes == -(-iters // T)     # every pass did work (no early stop)


@pytest.mark.parametrize("K", [1, 4, 10])
def test_to_tolerance_same_stop(sor, ctx, K):
    """Stops at the same checked iteration with the same change and grid."""
    n = 40
    g = random_small(41, n, with_f=True)
    for br, bc in ((8, 8), (5, 13)):
        for tol in (1e-2, 1e-5, 1e-9):
            ref = oracle.blockpar_f64(g.u0, g.bdy, g.f, 1.0, br, bc, tol, 50000, K, hist=True)
            _say(f"blockpar {br}x{bc} K={K} tol={tol} ref_it={ref.iterations}")
            assert ref.status == oracle.OK
            res, u = run(sor, ctx, g, br, bc, 1.0, tol, 50000, K)
            assert res.status == sor.OK and res.converged
            assert res.iterations == ref.iterations
            assert res.final_max_delta == ref.final_max_delta
            assert_bitwise(u, ref.u, f"u tol={tol}")
            assert_bitwise(np.array(res.hist), ref.mhist, f"hist tol={tol}")


@pytest.mark.parametrize("T", [2, 3, 5, 8])
@pytest.mark.parametrize("K", [1, 3, 7])
@pytest.mark.parametrize("bc", [11, 10])
def test_stop_inside_a_pass(sor, ctx, T, K, bc):
    """Checks that fall inside a pass: the pass is redone up to the stop from
    its input grid, so the result is the stopping iteration's (blocks of odd
    and of even width, which run different kernels)."""
    n = 70
    g = random_small(77 + T, n, with_f=False)
    ctx.set_variant_tiling(sor.ORDER_BLOCK_PARALLEL, T, 0)
    ref = oracle.blockpar_f64(g.u0, g.bdy, None, 1.1, 9, bc, 1e-4, 100000, K, hist=True)
    assert ref.status == oracle.OK
    res, u = run(sor, ctx, g, 9, bc, 1.1, 1e-4, 100000, K)
    assert (res.status, res.iterations) == (sor.OK, ref.iterations)
    assert res.final_max_delta == ref.final_max_delta
    assert_bitwise(u, ref.u, f"u T={T} K={K}")


def test_max_iters_not_multiple_of_k(sor, ctx):
    n = 33
    g = random_small(5, n, with_f=False)
    ref = oracle.blockpar_f64(g.u0, g.bdy, None, 1.2, 4, 6, 1e-14, 57, 10)
    res, u = run(sor, ctx, g, 4, 6, 1.2, 1e-14, 57, 10, hist=False)
    assert res.status == sor.NOT_CONVERGED and ref.status == oracle.NOT_CONVERGED
    assert res.iterations == 57 and res.final_max_delta == ref.final_max_delta
    assert_bitwise(u, ref.u, "u")


def test_limits_match_the_other_solvers(sor, ctx):
    """Blocks covering the grid give solve_f64's result, one-cell blocks the
    Jacobi ordering's (both on the GPU, bit for bit)."""
    n = 150
    g = random_small(15, n, with_f=True, nonzero_u0=True)
    res, u = run(sor, ctx, g, n, n + 3, 1.6, 0.0, 21, 1)
    u2 = dev(g.u0)
    r2 = sor.solve_f64(u2, dev(g.bdy), dev(g.f), 1.6, 0.0, 21, 1, hist=True, ctx=ctx)
    assert_bitwise(u, u2.cpu().numpy(), "one block vs red-black")
    assert_bitwise(np.array(res.hist), np.array(r2.hist), "one block vs red-black hist")
    res, u = run(sor, ctx, g, 1, 1, 0.9, 0.0, 21, 1)
    u3 = dev(g.u0)
    r3 = sor.solve_variant_f64(sor.ORDER_JACOBI, u3, dev(g.bdy), dev(g.f), 0.9, 0.0, 21, 1,
                               hist=True, ctx=ctx)
    assert_bitwise(u, u3.cpu().numpy(), "one-cell blocks vs Jacobi")
    assert_bitwise(np.array(res.hist), np.array(r3.hist), "one-cell blocks vs Jacobi hist")


def test_block_sides_beyond_the_grid(sor, ctx):
    """Block sides up to the largest int32 behave as sides of n (one block
    row or column): bit for bit the oracle, and red-black for both."""
    n = 90
    g = random_small(91, n, with_f=True, nonzero_u0=True)
    big = 2**31 - 1
    for br, bc in ((big, big), (big, 7), (8, big)):
        _say(f"blockpar blocks {br}x{bc} n={n}")
        check(sor, ctx, g, br, bc, 1.3, 12, f"{br}x{bc}")


def test_bench_grid_4096(sor, ctx):
    """The 4096^2 bench grid with 128 x 128 blocks, 6 iterations at the
    default tiling, whole grid compared."""
    g = laplace_random_boundary(4096)
    _say("blockpar 4096 oracle")
    ref = oracle.blockpar_f64(g.u0, g.bdy, None, 1.0, 128, 128, 0.0, 6, 1, hist=True)
    _say("blockpar 4096 gpu")
    res, u = run(sor, ctx, g, 128, 128, 1.0, 0.0, 6, 1)
    assert_bitwise(u, ref.u, "u 4096")
    assert_bitwise(np.array(res.hist), ref.mhist, "hist 4096")


@pytest.mark.parametrize("n,scale,T", [(37, 0.3, 1), (37, 0.3, 4), (130, 0.35, 8)])
def test_overflow_during_solve_reported(sor, ctx, n, scale, T):
    """Finite inputs whose iterates overflow between two checks (K = 10):
    ENONFINITE by the end of the pass holding the oracle's first infinite
    change, with the same changes up to it."""
    top = float(np.finfo(np.float64).max)
    g = Grid(n, np.zeros((n, n)), np.full(4 * n, scale * top), None, 1.0)
    ref = oracle.blockpar_f64(g.u0, g.bdy, None, 1.0, 6, 5, 0.0, 100, 10, hist=True)
    assert ref.status == oracle.ENONFINITE
    first_bad = ref.iterations
    ctx.set_variant_tiling(sor.ORDER_BLOCK_PARALLEL, T, 0)
    _say(f"blockpar overflow n={n} T={T} first_bad={first_bad}")
    res, _ = run(sor, ctx, g, 6, 5, 1.0, 0.0, 100, 10)
    assert res.status == sor.ENONFINITE and not res.converged, res
    assert first_bad <= res.iterations < first_bad + T, res.iterations
    assert_bitwise(res.hist[:first_bad], ref.mhist, "changes up to the overflow")


def test_argument_errors(sor, ctx):
    n = 20
    g = random_small(9, n, with_f=False)
    for br, bc in ((0, 4), (4, 0), (-1, 5)):
        with pytest.raises(sor.SorError) as e:
            run(sor, ctx, g, br, bc, 1.0, 0.0, 5, 1)
        assert e.value.status == sor.EINVAL
    with pytest.raises(sor.SorError) as e:
        sor.solve_variant_f64(sor.ORDER_BLOCK_PARALLEL, dev(g.u0), dev(g.bdy), None, 1.0,
                              0.0, 5, 1, ctx=ctx)
    assert e.value.status == sor.EINVAL
    with pytest.raises(sor.SorError):
        ctx.set_variant_tiling(sor.ORDER_BLOCK_PARALLEL, 9, 0)
    bdy = g.bdy.copy()
    bdy[7] = np.nan
    u = dev(g.u0)
    r = sor.solve_blockpar_f64(u, dev(bdy), 4, 4, None, 1.0, 1e-6, 50, 1, ctx=ctx)
    assert r.status == sor.ENONFINITE


@pytest.mark.parametrize("n", [1, 130])
def test_nan_from_finite_operands_reported(sor, ctx, n):
    """A NaN made from finite operands ((+inf) + (-inf) in a neighbour sum),
    whose change the running maximum drops: ENONFINITE like the oracle, at
    every depth (the passes check every interior cell they store)."""
    from test_nonfinite_gpu import interior_cross, opposite_boundary
    g = opposite_boundary(1, 64) if n == 1 else interior_cross(n, 64)
    for br, bc in ((1, 1), (4, 6), (n, n)):
        ref = oracle.blockpar_f64(g.u0, g.bdy, None, 1.0, br, bc, 0.0, 30, 10, hist=True)
        assert ref.status == oracle.ENONFINITE and ref.iterations == 1
        for T in (1, 3, 5, 8):
            ctx.set_variant_tiling(sor.ORDER_BLOCK_PARALLEL, T, 0)
            _say(f"blockpar nan-from-finite n={n} blocks {br}x{bc} T={T}")
            res, _ = run(sor, ctx, Grid(n, g.u0, g.bdy, None, 1.0), br, bc, 1.0, 0.0, 30, 10)
            assert res.status == sor.ENONFINITE and not res.converged, (T, res)
            assert 1 <= res.iterations <= T, (T, res.iterations)


def test_largest_side_sampled_windows(sor):
    """n = 65536 (two 34 GB working grids), 7 x 7 blocks, 2 iterations.  An
    iteration moves information by at most two cells (a black cell reads red
    values that read black ones), so the oracle on a window whose ring is
    frozen at the initial values is exact more than 2k cells inside it; the
    windows start at multiples of 7 with an even sum of offsets, so they see
    the same blocks and colours as the whole grid (65513 = 7 x 9359 puts the
    last windows against the south and east edges)."""
    n, k, blk = 65536, 2, 7
    rw = 12
    m = 2 * rw - 1
    core = slice(2 * k + 1, m - (2 * k + 1))
    ctx = sor.Context(0)
    try:
        rng = np.random.default_rng(65539)
        bdy = rng.uniform(0.0, 100.0, size=4 * n)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(23)
        _say("blockpar n=65536: filling u0 on the device")
        u = torch.rand((n, n), dtype=torch.float64, device="cuda", generator=gen) * 100.0
        last = n + 1 - 2 * rw                      # 65513, a multiple of 7, odd
        corners = [(0, 0), (0, 65506), (last, last), (65506, 0), (32760, 32774),
                   (1001, 7), (14, 31010), (40005, 7)]
        for a, b in corners:
            assert a % blk == 0 and b % blk == 0 and (a + b) % 2 == 0 and a <= last and b <= last
        before = {}
        for a, b in corners:
            lo_i, lo_j = max(a - 1, 0), max(b - 1, 0)
            before[(a, b)] = u[lo_i:a + 2 * rw, lo_j:b + 2 * rw].cpu().numpy().copy()
        _say("blockpar n=65536: solving")
        res = sor.solve_blockpar_f64(u, torch.tensor(bdy, dtype=torch.float64, device="cuda"),
                                     blk, blk, None, 1.3, 0.0, k, 1, hist=False, ctx=ctx)
        assert res.status == sor.NOT_CONVERGED and res.iterations == k

        def val_fn(blk_arr, lo_i, lo_j):
            def val(i, j):
                if i == 0:
                    return bdy[j - 1]
                if i == n + 1:
                    return bdy[n + j - 1]
                if j == 0:
                    return bdy[2 * n + i - 1]
                if j == n + 1:
                    return bdy[3 * n + i - 1]
                return blk_arr[i - 1 - lo_i, j - 1 - lo_j]
            return val

        for a, b in corners:
            _say(f"blockpar window at ({a}, {b})")
            lo_i, lo_j = max(a - 1, 0), max(b - 1, 0)
            val = val_fn(before[(a, b)], lo_i, lo_j)
            w0 = np.array([[val(a + 1 + r, b + 1 + c) for c in range(m)] for r in range(m)])
            wb = np.concatenate([[val(a, b + 1 + c) for c in range(m)],
                                 [val(a + 2 * rw, b + 1 + c) for c in range(m)],
                                 [val(a + 1 + r, b) for r in range(m)],
                                 [val(a + 1 + r, b + 2 * rw) for r in range(m)]])
            ref = oracle.blockpar_f64(w0, wb, None, 1.3, blk, blk, 0.0, k, 1)
            got = u[a:a + m, b:b + m].cpu().numpy()
            assert np.array_equal(got[core, core].view(np.uint64),
                                  ref.u[core, core].view(np.uint64)), (a, b)
        del u
    finally:
        ctx.close()
        torch.cuda.empty_cache()
