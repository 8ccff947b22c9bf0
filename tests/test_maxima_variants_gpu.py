"""Red-black passes that form only the maxima the stopping rule reads.

A pass of depth T applies iterations it0+1 .. it0+T.  When the check
interval K is at least T the pass holds at most one check iteration, and the
library launches a variant of the pass that forms that iteration's largest
change alone (or none at all); every iteration's change is formed when a
pass holds several checks or when the caller asks for the per-iteration
history.  These tests run solves without the history, so that the variants
run, at depths 6 and 7 (the ones with variants) with checks placed at every
position of a pass, and compare the stop iteration, the reported change and
the grid with the oracle bit for bit.  They also pin the non-finite rule the
passes follow: only a non-finite value is reported as such, while a change
that overflows between two finite values is an ordinary large change, as
Algorithm 1 counts it.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import Grid, random_small

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


def dev(a, dtype):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dtype,
                                               device="cuda")


def bits_of(a):
    a = np.asarray(a)
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def reference(g, bits, tol, iters, K, hist=False):
    if bits == 64:
        return oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, tol, iters, K, hist=hist)
    f = None if g.f is None else g.f.astype(np.float32)
    return oracle.sor_f32(g.u0.astype(np.float32), g.bdy.astype(np.float32), f, g.omega,
                          tol, iters, K, hist=hist)


def gpu(sor, ctx, g, bits, tol, iters, K, hist=False):
    dtype = torch.float64 if bits == 64 else torch.float32
    u = dev(g.u0, dtype)
    fn = sor.solve_f64 if bits == 64 else sor.solve_f32
    res = fn(u, dev(g.bdy, dtype), dev(g.f, dtype), g.omega, tol, iters, K, hist=hist,
             ctx=ctx)
    return res, u.cpu().numpy()


def scalar_bits(x, bits):
    return np.array([x], dtype=np.float64 if bits == 64 else np.float32).view(
        np.uint64 if bits == 64 else np.uint32)[0]


# Check intervals coprime to the depth: the checks K, 2K, ... T*K fall on
# every position 0 .. T-1 of a pass of depth T.
CASES = [(6, 7, 32), (7, 10, 40), (7, 10, 94)]


@pytest.mark.parametrize("T,K,seg", CASES)
@pytest.mark.parametrize("with_f", [False, True])
@pytest.mark.parametrize("bits", [64, 32])
def test_stop_at_every_position_of_a_pass(sor, ctx, bits, with_f, T, K, seg):
    n = 130
    g = random_small(11 + T, n, with_f=with_f, omega=1.0)
    full = reference(g, bits, 0.0, T * K, K, hist=True)
    ctx.set_tiling(bits, T, seg)
    covered = set()
    for m in range(1, T + 1):
        it = m * K
        mk = full.mhist[it - 1]
        earlier = [full.mhist[j * K - 1] for j in range(1, m)]
        tol = float(np.nextafter(mk, np.inf))
        if bits == 32:
            tol = float(np.nextafter(np.float32(mk), np.float32(np.inf)))
        if earlier and min(earlier) < tol:
            continue                       # an earlier check would pass first
        ref = reference(g, bits, tol, 10 * T * K, K)
        assert ref.status == oracle.OK and ref.iterations == it, (m, ref.iterations)
        pos = (it - 1) % T
        _say(f"maxima variant bits={bits} f={with_f} T={T} K={K} seg={seg} stop={it} pos={pos}")
        res, u = gpu(sor, ctx, g, bits, tol, 10 * T * K, K)
        assert res.status == sor.OK and res.converged, (it, res)
        assert res.iterations == it, (it, res.iterations)
        assert scalar_bits(res.final_max_delta, bits) == scalar_bits(ref.final_max_delta, bits), \
            (it, res.final_max_delta, ref.final_max_delta)
        assert np.array_equal(bits_of(u), bits_of(ref.u)), f"grid after stop at {it}"
        covered.add(pos)
    assert covered == set(range(T)), sorted(covered)


@pytest.mark.parametrize("T,seg", [(6, 32), (7, 40)])
@pytest.mark.parametrize("K", [3, 9, 20])
@pytest.mark.parametrize("bits", [64, 32])
def test_fixed_iterations_without_history(sor, ctx, bits, K, T, seg):
    """K < T (several checks per pass: every maximum formed), K > T (passes
    with one check and passes with none), and a last pass cut short by the
    iteration limit: final grid and last checked change as the oracle's."""
    n = 170
    g = random_small(23, n, with_f=True)
    iters = 5 * T + 4
    ref = reference(g, bits, 0.0, iters, K)
    ctx.set_tiling(bits, T, seg)
    _say(f"fixed iterations bits={bits} K={K} T={T}")
    res, u = gpu(sor, ctx, g, bits, 0.0, iters, K)
    assert res.status == sor.NOT_CONVERGED and res.iterations == iters
    assert scalar_bits(res.final_max_delta, bits) == scalar_bits(ref.final_max_delta, bits)
    assert np.array_equal(bits_of(u), bits_of(ref.u))


@pytest.mark.parametrize("bits", [64, 32])
def test_automatic_tiling_to_convergence(sor, ctx, bits):
    """The automatic depth and segment rows (from the occupancy of the
    variants), checks every 10 iterations and a stop found by the oracle."""
    n = 300
    g = random_small(31, n, with_f=False)
    tol = 1e-6 if bits == 64 else 1e-3
    ref = reference(g, bits, tol, 20000, 10)
    assert ref.status == oracle.OK
    _say(f"automatic tiling bits={bits} stop={ref.iterations}")
    res, u = gpu(sor, ctx, g, bits, tol, 20000, 10)
    assert res.status == sor.OK and res.iterations == ref.iterations
    assert scalar_bits(res.final_max_delta, bits) == scalar_bits(ref.final_max_delta, bits)
    assert np.array_equal(bits_of(u), bits_of(ref.u))


def overflowing_change():
    """One interior cell at +1e308 with a boundary at -5.25e306: its first
    update lands at about -1e308 (omega 1.9), so the change, 2e308, is above
    the largest double while both values are finite; the cell then contracts
    to a quarter of the boundary sum, its error shrinking by 0.9 per
    iteration."""
    return Grid(1, np.full((1, 1), 1e308), np.full(4, -5.25e306), None, 1.9)


@pytest.mark.parametrize("K", [1, 10])
@pytest.mark.parametrize("hist", [False, True])
def test_change_overflow_between_finite_values(sor, ctx, hist, K):
    """The changes of the first two iterations overflow; the solve runs on
    to the stop (changes below 1e300) exactly as the oracle's."""
    g = overflowing_change()
    ref = reference(g, 64, 1e300, 2000, K, hist=True)
    assert np.isinf(ref.mhist[0]) and np.isfinite(ref.u).all()
    assert ref.status == oracle.OK
    for T, seg in [(1, 8), (6, 32), (7, 40), (0, 0)]:
        _say(f"overflowing change hist={hist} K={K} T={T}")
        ctx.set_tiling(64, T, seg)                 # (0, 0): automatic
        res, u = gpu(sor, ctx, g, 64, 1e300, 2000, K, hist=hist)
        assert res.status == sor.OK and res.iterations == ref.iterations, (T, res)
        assert scalar_bits(res.final_max_delta, 64) == scalar_bits(ref.final_max_delta, 64), T
        assert np.array_equal(bits_of(u), bits_of(ref.u)), T
        if hist:
            it = ref.iterations
            assert np.array_equal(bits_of(np.array(res.hist)[:it]), bits_of(ref.mhist[:it])), T
