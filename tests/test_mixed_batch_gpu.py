"""GPU parity of mixed-precision batched solves and of the request server.

Grids and requests that pass no inner iteration count get the library's
default (n/2 rounded up to a multiple of 6); the oracle's default is the same
count.  Each
grid, whether solved in a batch or served among other requests, must equal
the CPU oracle's defect-correction solve of that grid alone bit for bit at
the same number of corrections (the inner sweeps, casts and corrections are
exactly rounded; only the stopping test's norm sums differ in order)."""
import time

import numpy as np
import pytest

import oracle
from workloads import omega_opt, poisson_manufactured, random_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def grids_for(seed, sizes):
    out = []
    for k, n in enumerate(sizes):
        g = random_small(seed * 100 + k, n, with_f=(k % 3 != 0), nonzero_u0=(k % 2 == 0))
        if k % 4 == 1:
            g = poisson_manufactured(n, seed=seed + k)
        out.append(g)
    return out


@pytest.mark.parametrize("bits,odd", [(32, False), (16, False), (32, True)])
def test_mixed_batch_fixed_corrections_bitwise(sor, ctx, bits, odd):
    """Two corrections per grid with the default inner count (a multiple of
    the kernel's fixed depth), and with counts that are not (the run-time
    depth kernel: 2n + 1, and 1, 2, 3 on the smallest grids)."""
    grids = grids_for(1, [1, 4, 33, 64, 100, 130, 7, 250])
    outer = 2
    inner = [2 * g.n + 1 if g.n > 4 else g.n + 1 for g in grids] if odd else [None] * len(grids)
    us = [dev(g.u0) for g in grids]
    specs = [sor.MixedSpec(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 0.0, outer, m or 0)
             for u, g, m in zip(us, grids, inner)]
    res = sor.batch_solve_mixed(specs, bits, ctx=ctx)
    for k, (g, r, u) in enumerate(zip(grids, res, us)):
        ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, outer, bits, inner[k])
        assert r.outer_steps == ref.outer_steps == outer, (k, r)
        assert bitwise(u.cpu().numpy(), ref.u), (k, g.n)
        assert abs(r.rel_residual - ref.rel_residual) <= 1e-9 * ref.rel_residual + 1e-300


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_mixed_batch_shallower_context_depth(sor, ctx, depth):
    """A depth set on the context below the fixed depth of the persistent
    kernel: the inner passes must still apply exactly the counted iterations
    (the run-time-depth kernel), so the result is the oracle's bit for bit,
    with default inner counts and with odd ones."""
    ctx.set_tiling(32, depth, 0)
    grids = grids_for(5, [4, 33, 100, 130, 250, 520])
    for inner in (None, 13):
        us = [dev(g.u0) for g in grids]
        specs = [sor.MixedSpec(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 0.0, 2, inner or 0)
                 for u, g in zip(us, grids)]
        res = sor.batch_solve_mixed(specs, 32, ctx=ctx)
        for k, (g, r, u) in enumerate(zip(grids, res, us)):
            ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, 2, 32, inner)
            assert r.outer_steps == ref.outer_steps == 2, (k, r)
            assert bitwise(u.cpu().numpy(), ref.u), (depth, inner, k, g.n)


@pytest.mark.parametrize("bits,tol", [(32, 1e-11), (16, 1e-9)])
def test_mixed_batch_to_tolerance(sor, ctx, bits, tol):
    grids = grids_for(2, [20, 63, 127, 90, 200])
    us = [dev(g.u0) for g in grids]
    specs = [sor.MixedSpec(u, dev(g.bdy), dev(g.f), None, tol, 0.0, 40, 0)
             for u, g in zip(us, grids)]
    res = sor.batch_solve_mixed(specs, bits, ctx=ctx)
    for k, (g, r, u) in enumerate(zip(grids, res, us)):
        ref = oracle.mixed(g.u0, g.bdy, g.f, omega_opt(g.n), tol, 40, bits)
        assert ref.converged and r.converged, (k, r, ref.relhist)
        assert r.outer_steps == ref.outer_steps, (k, r.outer_steps, ref.outer_steps)
        assert r.rel_residual <= tol
        assert bitwise(u.cpu().numpy(), ref.u), k


def test_mixed_batch_correction_stop_rule(sor, ctx):
    grids = grids_for(3, [40, 80, 120])
    us = [dev(g.u0) for g in grids]
    specs = [sor.MixedSpec(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 1e-8, 30, 0)
             for u, g in zip(us, grids)]
    res = sor.batch_solve_mixed(specs, 32, ctx=ctx)
    for k, (g, r, u) in enumerate(zip(grids, res, us)):
        ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, 30, 32, corr_tol=1e-8)
        assert ref.converged and r.converged
        assert r.outer_steps == ref.outer_steps
        assert r.final_max_delta == ref.last_correction
        assert bitwise(u.cpu().numpy(), ref.u), k


def _nonfinite_cases(n, seed):
    """(boundary, source) pairs with no finite solution or with 2-norms that
    overflow: a NaN in the source, an infinite boundary value, entries of
    about 1e200."""
    g = random_small(seed, n, with_f=True)
    nan_f = g.f.copy()
    nan_f[n // 2, 1] = np.nan
    inf_b = g.bdy.copy()
    inf_b[n + 2] = np.inf
    return [(g.bdy, nan_f), (inf_b, g.f), (g.bdy * 1e200, None)]


@pytest.mark.parametrize("bits", [32, 16])
def test_mixed_nonfinite_data_reported(sor, ctx, bits):
    """Single mixed solves and a mixed batch: data with a NaN, an infinity or
    overflowing norms ends with ENONFINITE before any correction, as in the
    oracle; the finite grids of the same batch are still the oracle's bit for
    bit."""
    n = 40
    cases = _nonfinite_cases(n, 61)
    for k, (b, f) in enumerate(cases):
        ref = oracle.mixed(np.zeros((n, n)), b, f, omega_opt(n), 1e-9, 40, bits, 2 * n)
        assert ref.status == oracle.ENONFINITE and ref.outer_steps == 0, k
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        r = sor.solve_mixed(u, dev(b), dev(f), omega_opt(n), 1e-9, 40, bits, 2 * n, ctx=ctx)
        assert r.status == sor.ENONFINITE and r.outer_steps == 0, (k, r)
    good = grids_for(6, [30, 57, 90])
    grids = [(g.bdy, g.f, g.u0) for g in good] + [(b, f, np.zeros((n, n))) for b, f in cases]
    us = [dev(u0) for _, _, u0 in grids]
    specs = [sor.MixedSpec(u, dev(b), dev(f), None, 1e-9, 0.0, 40, 0)
             for u, (b, f, _) in zip(us, grids)]
    res = sor.batch_solve_mixed(specs, bits, ctx=ctx)
    for k, (g, r, u) in enumerate(zip(good, res, us)):
        ref = oracle.mixed(g.u0, g.bdy, g.f, omega_opt(g.n), 1e-9, 40, bits)
        assert ref.converged and r.converged, (k, r)
        assert r.outer_steps == ref.outer_steps
        assert bitwise(u.cpu().numpy(), ref.u), k
    for k in range(len(good), len(grids)):
        assert res[k].status == sor.ENONFINITE and res[k].outer_steps == 0, (k, res[k])


def test_server_nonfinite_request_reported(sor):
    """A request with non-finite data completes with ENONFINITE; the requests
    around it still equal the oracle's standalone solves bit for bit."""
    n = 40
    cases = _nonfinite_cases(n, 62)
    good = [random_small(700 + k, m, with_f=True) for k, m in enumerate([24, 50, 33])]
    reqs = [(g.bdy, g.f) for g in good[:2]] + cases + [(good[2].bdy, good[2].f)]
    srv = sor.Server(0, inner_bits=32, hbm_budget=24 << 20, max_slots=3, slice_ms=0.3)
    try:
        tickets = [srv.submit(b, f, None, 0.0, 1e-9, 0.0, 40, 0) for b, f in reqs]
        done = {}
        t_end = time.time() + 120
        while len(done) < len(tickets) and time.time() < t_end:
            for t in tickets:
                if t not in done:
                    c = srv.poll(t, wait_ms=5.0)
                    if c is not None:
                        done[t] = c
        assert len(done) == len(tickets), srv.stats()
    finally:
        srv.close()
    for k in range(2, 2 + len(cases)):
        assert done[tickets[k]].status == sor.ENONFINITE, (k, done[tickets[k]].result)
    for t, g in zip([tickets[0], tickets[1], tickets[-1]], good):
        c = done[t]
        ref = oracle.mixed(np.zeros((g.n, g.n)), g.bdy, g.f, omega_opt(g.n), 1e-9, 40, 32)
        assert c.status == sor.OK and ref.converged, (g.n, c.result)
        assert bitwise(c.u, ref.u), g.n


@pytest.mark.parametrize("bits", [32, 16])
def test_server_results_equal_standalone(sor, bits):
    """A stream of requests through a small server (few slots, small memory
    budget, short time slices, so requests wait, pause and resume): every
    result equals the oracle's standalone solve bit for bit."""
    rng = np.random.default_rng(7)
    sizes = [int(rng.choice([16, 50, 100, 130, 200])) for _ in range(12)]
    grids = [random_small(500 + k, n, with_f=True) for k, n in enumerate(sizes)]
    tol = 1e-9 if bits == 32 else 1e-8
    srv = sor.Server(0, inner_bits=bits, hbm_budget=24 << 20, max_slots=3, slice_ms=0.3)
    try:
        tickets = []
        for g in grids:
            tickets.append(srv.submit(g.bdy, g.f, None, 0.0, tol, 0.0, 40, 0))
            time.sleep(0.002)
        done = {}
        t_end = time.time() + 120
        while len(done) < len(tickets) and time.time() < t_end:
            for t in tickets:
                if t not in done:
                    c = srv.poll(t, wait_ms=5.0)
                    if c is not None:
                        done[t] = c
        assert len(done) == len(tickets), srv.stats()
        st = srv.stats()
        assert st["completed"] == len(tickets) and st["launches"] > 1, st
    finally:
        srv.close()
    for t, g in zip(tickets, grids):
        c = done[t]
        ref = oracle.mixed(np.zeros((g.n, g.n)), g.bdy, g.f, omega_opt(g.n), tol, 40, bits)
        assert c.status == sor.OK and ref.converged, (g.n, c.result)
        assert c.result.outer_steps == ref.outer_steps
        assert bitwise(c.u, ref.u), g.n
        assert c.submit_s <= c.admit_s <= c.done_s


def test_server_admission_budget_and_no_head_of_line_blocking(sor):
    """A budget that holds one large request or a few small ones: a large
    request that cannot be admitted while another large one is resident does
    not hold back the small requests submitted after it (they finish first),
    the bytes held never exceed the budget, and every result equals the
    oracle's standalone solve bit for bit."""
    from paper_1401_0763_amd import Server
    big = [random_small(800 + k, 300, with_f=True) for k in range(2)]
    small = [random_small(810 + k, 40, with_f=True) for k in range(6)]
    budget = 8 << 20            # one n = 300 request (5.9 MiB) and four n = 40 (0.5 MiB each)
    srv = Server(0, inner_bits=32, hbm_budget=budget, max_slots=8, slice_ms=0.5)
    try:
        order = [big[0], big[1]] + small
        tickets = [srv.submit(g.bdy, g.f, None, 0.0, 1e-9, 0.0, 40, 0) for g in order]
        done = {}
        t_end = time.time() + 120
        while len(done) < len(tickets) and time.time() < t_end:
            for t in tickets:
                if t not in done:
                    c = srv.poll(t, wait_ms=2.0)
                    if c is not None:
                        done[t] = c
        assert len(done) == len(tickets), srv.stats()
        mem = srv.memory()
    finally:
        srv.close()
    assert mem["budget"] == budget and 0 < mem["peak"] <= budget and mem["in_use"] == 0, mem
    # The first four small requests fit beside the first large one as soon as
    # they arrive; the second large one waits for the first to leave.
    second_big = done[tickets[1]]
    assert second_big.admit_s >= done[tickets[0]].done_s - 1e-3
    for t in tickets[2:6]:
        assert done[t].admit_s <= second_big.admit_s, (done[t].admit_s, second_big.admit_s)
    for t, g in zip(tickets, order):
        ref = oracle.mixed(np.zeros((g.n, g.n)), g.bdy, g.f, omega_opt(g.n), 1e-9, 40, 32)
        assert done[t].status == sor.OK and bitwise(done[t].u, ref.u), g.n
