"""GPU parity of batched solves: every grid of a batch must equal the CPU
oracle's solve of that grid alone, bit for bit, with the same stopping
iteration; a grid's result must not depend on the rest of the batch."""
import sys

import numpy as np
import pytest

import oracle
from workloads import batch_grids, omega_opt, random_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


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


def bitwise(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def mixed_specs(seed, count):
    """Grids of varied size, source, omega, tolerance, cadence and limit."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.choice([1, 2, 3, 7, 16, 33, 64, 65, 100, 127, 200, 257]))
        g = random_small(int(rng.integers(1 << 30)), n, with_f=bool(k % 2),
                         nonzero_u0=bool(k % 3 == 0))
        g.omega = float(rng.choice([omega_opt(n), 1.0, 0.376, 1.5]))
        g.tol = float(rng.choice([1e-3, 1e-6, 1e-9, 0.0]))
        g.check_every = int(rng.choice([1, 3, 10]))
        g.max_iters = int(rng.choice([1, 7, 50, 400, 2000]))
        out.append(g)
    return out


def run_batch(sor, ctx, grids):
    us = [dev(g.u0) for g in grids]
    specs = [sor.GridSpec(u, dev(g.bdy), dev(g.f), g.omega, g.tol, g.max_iters,
                          g.check_every) for u, g in zip(us, grids)]
    res = sor.batch_solve_f64(specs, ctx=ctx)
    return res, [u.cpu().numpy() for u in us]


def check_against_oracle(grids, res, us):
    for k, (g, r, u) in enumerate(zip(grids, res, us)):
        ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, g.tol, g.max_iters, g.check_every)
        assert r.status == ref.status, (k, g.n, r, ref.status)
        assert r.iterations == ref.iterations, (k, g.n, r.iterations, ref.iterations)
        if ref.status == oracle.OK:
            assert r.final_max_delta == ref.final_max_delta, (k, g.n)
        assert bitwise(u, ref.u), (k, g.n, np.abs(u - ref.u).max())


@pytest.mark.parametrize("seed,count", [(1, 24), (2, 40)])
def test_batch_matches_oracle_per_grid(sor, ctx, seed, count):
    grids = mixed_specs(seed, count)
    _say(f"batch seed={seed} count={count} sizes={[g.n for g in grids]}")
    res, us = run_batch(sor, ctx, grids)
    check_against_oracle(grids, res, us)


def test_batch_graph_replay_and_mix_invariance(sor, ctx):
    grids = mixed_specs(3, 16)
    res1, us1 = run_batch(sor, ctx, grids)          # records the graph
    res2, us2 = run_batch(sor, ctx, grids)          # replays it
    for a, b in zip(us1, us2):
        assert bitwise(a, b)
    check_against_oracle(grids, res2, us2)
    # the same grid alone gives the same bits
    for k in (0, 5, 11):
        r, u = run_batch(sor, ctx, [grids[k]])
        assert r[0].iterations == res1[k].iterations
        assert bitwise(u[0], us1[k])


def test_batch_log_uniform_sizes_to_tolerance(sor, ctx):
    """A smaller draw of the batched workload: sides log-uniform in [64, 256],
    f on odd grids, omega_opt, tol 1e-8 checked every iteration."""
    grids = batch_grids(count=24, lo=64, hi=256, seed=4, tol=1e-8)
    for g in grids:
        g.max_iters = 20000
    res, us = run_batch(sor, ctx, grids)
    assert all(r.converged for r in res)
    check_against_oracle(grids, res, us)


def test_batch_nonfinite_grid_reported(sor, ctx):
    grids = mixed_specs(4, 6)
    for g in grids:
        g.max_iters = 50
    grids[2].bdy = grids[2].bdy.copy()
    grids[2].bdy[0] = np.inf
    us = [dev(g.u0) for g in grids]
    specs = [sor.GridSpec(u, dev(g.bdy), dev(g.f), g.omega, g.tol, g.max_iters,
                          g.check_every) for u, g in zip(us, grids)]
    res = sor.batch_solve_f64(specs, ctx=ctx)
    assert res[2].status == sor.ENONFINITE
    for k in (0, 1, 3, 4, 5):
        assert res[k].status in (sor.OK, sor.NOT_CONVERGED)


def test_batch_overflow_grid_reported(sor, ctx):
    """A grid whose finite iterates overflow between two checks (uniform
    boundary at 0.15 of the largest double, first infinite change at
    iteration 6) ends with ENONFINITE; the other grids of the batch are still
    the oracle's bit for bit."""
    from workloads import Grid
    n = 130
    top = float(np.finfo(np.float64).max)
    bad = Grid(n, np.zeros((n, n)), np.full(4 * n, 0.15 * top), None, omega_opt(n),
               tol=0.0, max_iters=50, check_every=10)
    ref = oracle.sor_f64(bad.u0, bad.bdy, None, bad.omega, 0.0, 50, 10)
    assert ref.status == oracle.ENONFINITE and ref.iterations == 6
    grids = mixed_specs(7, 6)
    grids[2] = bad
    _say(f"batch overflow sizes={[g.n for g in grids]}")
    res, us = run_batch(sor, ctx, grids)
    assert res[2].status == sor.ENONFINITE and not res[2].converged, res[2]
    assert 6 <= res[2].iterations < 6 + 8, res[2].iterations
    others = [k for k in range(len(grids)) if k != 2]
    check_against_oracle([grids[k] for k in others], [res[k] for k in others],
                         [us[k] for k in others])


def test_autotune_returns_supported_tiling_and_keeps_results(sor, ctx):
    T, seg = ctx.autotune(64, 300)
    assert 1 <= T <= 8 and 8 <= seg <= 1024
    g = random_small(55, 300, with_f=True)
    ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 0.0, 30, 1)
    u = dev(g.u0)
    sor.solve_f64(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 30, 1, ctx=ctx)
    assert bitwise(u.cpu().numpy(), ref.u)


def test_batch_autotune_returns_supported_tiling_and_keeps_results(sor, ctx):
    """The batched tuner records a tiling for the class of n = 100 only in the
    batched table; batches of that class still equal the oracle bit for bit,
    and a plain solve keeps its own tiling."""
    plain_before = ctx.tiling_for(64, 100)
    T, seg = ctx.autotune_batch(64, 100)
    # Batched FP64 passes have a fixed depth (7): only the tile height is
    # tuned.
    assert T == 7 and 16 <= seg <= 384
    assert ctx.tiling_for(64, 100) == plain_before
    grids = []
    for k in range(4):
        g = random_small(300 + k, 100, with_f=bool(k % 2))
        g.tol, g.max_iters, g.check_every = 1e-7, 3000, 1
        grids.append(g)
    res, us = run_batch(sor, ctx, grids)
    for g, r, u in zip(grids, res, us):
        ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, g.tol, g.max_iters, 1)
        assert r.iterations == ref.iterations and r.status == ref.status
        assert bitwise(u, ref.u)
