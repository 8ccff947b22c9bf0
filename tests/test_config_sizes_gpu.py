"""GPU parity at the workload sizes: batched grids of sides 512..1024 (with the
size rule's tiles and with batch-autotuned tiles), served requests of sides
1024..2048 in a mix, the 4096^2 mixed-precision solve, and the stop
iterations of the 4096^2 plain solves (to max |du| < 1e-8, and the paper's
own configuration of Sec. 4).

Every result is compared with the CPU oracle bit for bit: grids, final
changes and stop iterations.  The two 4096^2 stop-at-tolerance solves take
the oracle minutes, so their oracle results are stored in
tests/golden/oracle_4096_stops.json (written by make_oracle_4096.py next to
it, which calls only the oracle) and compared by SHA-256 of the grid."""
import hashlib
import json
import os
import struct
import time

import numpy as np
import pytest

import oracle
from workloads import (batch_grids, laplace_random_boundary, laplace_top_edge, omega_opt,
                       poisson_manufactured, random_grid)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_4096_stops.json")
THREADS = 8          # oracle workers (bitwise equal to one thread)


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sor():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1401_0763_amd as m
    return m


def dev(a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                               device="cuda")


def bitwise(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def c4_subset():
    """Twelve grids of side >= 512 and twenty smaller ones from the batched
    workload's draw (sides log-uniform in [64, 1024], seed 4), plus one grid
    of the largest side 1024."""
    gs = batch_grids(512, 64, 1024, seed=4)
    sel = [g for g in gs if g.n >= 512][:12] + [g for g in gs if g.n < 512][:20]
    sel.append(random_grid(np.random.default_rng(41), 1024, with_f=True))
    return sel


def _batch_vs_oracle(sor, ctx, grids, tol, iters, K):
    us = [torch.zeros((g.n, g.n), dtype=torch.float64, device="cuda") for g in grids]
    specs = [sor.GridSpec(u, dev(g.bdy), dev(g.f), g.omega, tol, iters, K)
             for u, g in zip(us, grids)]
    res = sor.batch_solve_f64(specs, ctx=ctx)
    for k, (g, r, u) in enumerate(zip(grids, res, us)):
        ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, tol, iters, K, threads=THREADS)
        assert (r.status, r.iterations) == (ref.status, ref.iterations), (k, g.n, r, ref.iterations)
        assert bits(r.final_max_delta) == bits(ref.final_max_delta), (k, g.n)
        assert bitwise(u.cpu().numpy(), ref.u), (k, g.n)


@pytest.mark.parametrize("tuned", [False, True])
def test_c4_grids_fixed_iterations(sor, tuned):
    """33 grids with sides up to 1024, 150 iterations each, checked every
    iteration, in one persistent launch: with the size rule's tiles (128 rows
    below n = 512, 384 above), then with tiles from the batched autotuner for
    the classes of n = 1024 and n = 700."""
    ctx = sor.Context(0)
    try:
        if tuned:
            for n in (1024, 700):
                T, seg = ctx.autotune_batch(64, n)
                _say(f"autotuned n={n}: T={T} seg={seg}")
        grids = c4_subset()
        _say(f"c4 subset: {len(grids)} grids, sides {min(g.n for g in grids)}.."
             f"{max(g.n for g in grids)}, tuned={tuned}")
        _batch_vs_oracle(sor, ctx, grids, 0.0, 150, 1)
    finally:
        ctx.close()


def test_c4_whole_batch_every_grid(sor):
    """The whole batched workload (512 grids, sides 64..1024, FP64 to max |du|
    < 1e-8 checked every iteration, then FP32 + FP64 refinement with two
    corrections of the default inner count) in one launch each: every grid's
    stop iteration, final change and values equal the oracle's standalone
    solve bit for bit."""
    grids = batch_grids(512, 64, 1024, seed=4, tol=1e-8)
    ctx = sor.Context(0)
    try:
        us = [torch.zeros((g.n, g.n), dtype=torch.float64, device="cuda") for g in grids]
        specs = [sor.GridSpec(u, dev(g.bdy), dev(g.f), g.omega, 1e-8, 200000, 1)
                 for u, g in zip(us, grids)]
        res = sor.batch_solve_f64(specs, ctx=ctx)
        um = [torch.zeros((g.n, g.n), dtype=torch.float64, device="cuda") for g in grids]
        mspecs = [sor.MixedSpec(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 0.0, 2, 0)
                  for u, g in zip(um, grids)]
        mres = sor.batch_solve_mixed(mspecs, 32, ctx=ctx)
        got = [u.cpu().numpy() for u in us]
        gotm = [u.cpu().numpy() for u in um]
    finally:
        ctx.close()
    t0 = time.time()
    for k, g in enumerate(grids):
        ref = oracle.sor_f64(g.u0, g.bdy, g.f, g.omega, 1e-8, 200000, 1, threads=16)
        assert (res[k].status, res[k].iterations) == (ref.status, ref.iterations), (k, g.n)
        assert bits(res[k].final_max_delta) == bits(ref.final_max_delta), (k, g.n)
        assert bitwise(got[k], ref.u), (k, g.n)
        mref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, 2, 32, threads=16)
        assert mres[k].outer_steps == mref.outer_steps == 2, (k, g.n)
        assert bitwise(gotm[k], mref.u), ("mixed", k, g.n)
        if k % 64 == 63:
            _say(f"whole batch: {k + 1} grids equal to the oracle ({time.time() - t0:.0f} s)")


def test_c4_large_grids_to_tolerance(sor):
    """Three grids of sides 802..1024 solved to max |du| < 1e-8 (checked every
    iteration) among small ones: stop iterations of several thousand, equal
    to the oracle's, with equal grids."""
    gs = c4_subset()
    big = [g for g in gs if g.n in (1024, 961, 802)]
    small = [g for g in gs if g.n < 200][:6]
    ctx = sor.Context(0)
    try:
        _batch_vs_oracle(sor, ctx, big + small, 1e-8, 200000, 1)
    finally:
        ctx.close()


def test_c4_mixed_batch_large_grids(sor):
    """The FP32 + FP64-refinement batch on grids of sides up to 1024: two
    corrections with the default inner count (about n/2) per grid, bit for
    bit."""
    gs = c4_subset()
    grids = [g for g in gs if g.n >= 512][:5] + [gs[-1]] + [g for g in gs if g.n < 512][:4]
    ctx = sor.Context(0)
    try:
        us = [torch.zeros((g.n, g.n), dtype=torch.float64, device="cuda") for g in grids]
        specs = [sor.MixedSpec(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 0.0, 2, 0)
                 for u, g in zip(us, grids)]
        res = sor.batch_solve_mixed(specs, 32, ctx=ctx)
        for k, (g, r, u) in enumerate(zip(grids, res, us)):
            ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, 2, 32, threads=THREADS)
            assert r.outer_steps == ref.outer_steps == 2, (k, g.n, r)
            assert bitwise(u.cpu().numpy(), ref.u), (k, g.n)
    finally:
        ctx.close()


def test_served_large_requests_in_a_mix(sor):
    """Requests of sides 1024..2048 (the upper half of the served workload's
    range) submitted among small ones to a server with room for only some of
    them at once: each result equals the oracle's standalone solve (two
    corrections, default inner count) bit for bit."""
    rng = np.random.default_rng(55)
    sizes = [1024, 96, 2048, 130, 1536, 64, 1200, 200]
    grids = [random_grid(rng, n, with_f=True) for n in sizes]
    srv = sor.Server(0, inner_bits=32, hbm_budget=400 << 20, max_slots=4, slice_ms=2.0)
    try:
        tickets = []
        for g in grids:
            tickets.append(srv.submit(g.bdy, g.f, None, 0.0, 0.0, 0.0, 2, 0))
            time.sleep(0.005)
        done = {}
        t_end = time.time() + 90
        while len(done) < len(tickets) and time.time() < t_end:
            for t in tickets:
                if t not in done:
                    c = srv.poll(t, wait_ms=5.0)
                    if c is not None:
                        done[t] = c
        assert len(done) == len(tickets), srv.stats()
    finally:
        srv.close()
    for t, g in zip(tickets, grids):
        c = done[t]
        ref = oracle.mixed(np.zeros((g.n, g.n)), g.bdy, g.f, omega_opt(g.n), 0.0, 2, 32,
                           threads=THREADS)
        assert c.status == sor.NOT_CONVERGED and c.result.outer_steps == 2, (g.n, c.result)
        assert bitwise(c.u, ref.u), g.n
        _say(f"served n={g.n}: bitwise equal to the oracle")


def test_c3_fp32_correction_at_4096(sor):
    """The 4096^2 Poisson problem of the mixed-precision workload (f = N(0,1)
    + 2 pi^2 sin sin, seed 3): one FP32 correction of 300 inner iterations,
    bit for bit against the oracle, with the same relative residuals."""
    g = poisson_manufactured(4096, seed=3)
    ctx = sor.Context(0)
    try:
        u = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
        r = sor.solve_mixed(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 1, 32, 300, hist=True,
                            ctx=ctx)
        got = u.cpu().numpy()
    finally:
        ctx.close()
    ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, 1, 32, 300, threads=THREADS)
    assert r.outer_steps == ref.outer_steps == 1
    assert bitwise(got, ref.u)
    assert np.allclose(r.hist, ref.relhist, rtol=1e-9, atol=0)


def test_binary16_limit_and_largest_size(sor):
    """binary16 inner storage is refused above n = 1024 by the single, batched
    and served forms; at n = 1024 one correction is the oracle's bit for bit
    and the default settings reach a relative residual of 1e-8 within 30
    corrections on the mixed-precision workload's problem at that size."""
    ctx = sor.Context(0)
    try:
        n = 1025
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        b = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
        with pytest.raises(sor.SorError) as e:
            sor.solve_mixed(u, b, None, 1.5, 1e-8, 3, 16, 0, ctx=ctx)
        assert e.value.status == sor.EINVAL
        with pytest.raises(sor.SorError) as e:
            sor.batch_solve_mixed([sor.MixedSpec(u, b, None, 1.5, 1e-8, 0.0, 3, 0)], 16, ctx=ctx)
        assert e.value.status == sor.EINVAL
        srv = sor.Server(0, inner_bits=16, hbm_budget=1 << 30, max_slots=2)
        try:
            with pytest.raises(sor.SorError):
                srv.submit(np.zeros(4 * n), None)
        finally:
            srv.close()
        g = poisson_manufactured(1024, seed=3)
        u = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
        r = sor.solve_mixed(u, dev(g.bdy), dev(g.f), g.omega, 0.0, 1, 16, 0, ctx=ctx)
        got = u.cpu().numpy()
        ref = oracle.mixed(g.u0, g.bdy, g.f, g.omega, 0.0, 1, 16, threads=THREADS)
        assert r.outer_steps == ref.outer_steps == 1
        assert bitwise(got, ref.u)
        u.zero_()
        r = sor.solve_mixed(u, dev(g.bdy), dev(g.f), g.omega, 1e-8, 30, 16, 0, hist=True,
                            ctx=ctx)
        _say(f"binary16 n=1024: {r.outer_steps} corrections, rel {r.rel_residual:.3e}")
        assert r.status == sor.OK and r.rel_residual <= 1e-8, r.hist
    finally:
        ctx.close()


@pytest.mark.parametrize("name", ["tol_1e-8", "paper"])
def test_4096_stop_iteration_equals_stored_oracle(sor, name):
    """4096^2 plain FP64 solves to a tolerance: the stop iteration, the final
    change and the whole grid equal the oracle's stored results."""
    with open(GOLDEN) as fh:
        case = next(c for c in json.load(fh)["cases"] if c["name"] == name)
    if name == "paper":
        g = laplace_top_edge(4096, top=1.0)
    else:
        g = laplace_random_boundary(4096, seed=2)
    assert case["omega"] == (0.376 if name == "paper" else g.omega)
    ctx = sor.Context(0)
    try:
        u = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
        r = sor.solve_f64(u, dev(g.bdy), None, case["omega"], case["tol"], case["max_iters"],
                          case["check_every"], ctx=ctx)
        got = u.cpu().numpy()
    finally:
        ctx.close()
    _say(f"{name}: stop at {r.iterations} (oracle {case['iterations']})")
    assert r.status == case["status"] and r.iterations == case["iterations"]
    assert f"{bits(r.final_max_delta):016x}" == case["final_max_delta_bits"]
    assert hashlib.sha256(np.ascontiguousarray(got).tobytes()).hexdigest() == case["u_sha256"]
    for i, j, hx in case["samples"]:
        assert f"{bits(float(got[i, j])):016x}" == hx
