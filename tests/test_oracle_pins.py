"""Pins of the CPU oracle against things other than itself.

Each test ties the oracle to a hand-worked example, a closed form, a textbook
special case solved by a different method (dense LU, DST-I diagonalisation,
separation of variables), an invariant of the discrete problem, or a library
routine.  A dropped term, a wrong sign or index, a transposed boundary edge or
the wrong phase order in the oracle breaks at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft

import oracle
from workloads import laplace_top_edge, manufactured_term, omega_opt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------------------
# Independent solvers of the discrete system A u = b (h*h-scaled 5-point)
# ---------------------------------------------------------------------------

def dense_system(n, bdy, f):
    """Assemble A (n^2 x n^2) and b from the stencil definition, cell by cell."""
    h = 1.0 / (n + 1)
    north, south, west, east = (bdy[0:n], bdy[n:2 * n], bdy[2 * n:3 * n],
                                bdy[3 * n:4 * n])
    N = n * n
    A = np.zeros((N, N))
    b = np.zeros(N)
    for i in range(n):          # i = 0 is the row next to the north edge
        for j in range(n):
            k = i * n + j
            A[k, k] = 4.0
            b[k] = h * h * f[i, j] if f is not None else 0.0
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    A[k, ii * n + jj] = -1.0
                elif ii < 0:
                    b[k] += north[j]
                elif ii >= n:
                    b[k] += south[j]
                elif jj < 0:
                    b[k] += west[i]
                else:
                    b[k] += east[i]
    return A, b


def dense_solve(n, bdy, f):
    A, b = dense_system(n, bdy, f)
    return np.linalg.solve(A, b).reshape(n, n)


def dst_solve(n, bdy, f):
    """Exact discrete solution via the DST-I, which diagonalises the Dirichlet
    5-point Laplacian: eigenvalues 4(sin^2(p pi h/2) + sin^2(q pi h/2))."""
    h = 1.0 / (n + 1)
    b = np.zeros((n, n)) if f is None else h * h * np.asarray(f, float).copy()
    b[0, :] += bdy[0:n]
    b[-1, :] += bdy[n:2 * n]
    b[:, 0] += bdy[2 * n:3 * n]
    b[:, -1] += bdy[3 * n:4 * n]
    p = np.arange(1, n + 1)
    s2 = np.sin(p * np.pi * h / 2.0) ** 2
    lam = 4.0 * (s2[:, None] + s2[None, :])
    bh = scipy.fft.dstn(b, type=1, norm="ortho")
    return scipy.fft.idstn(bh / lam, type=1, norm="ortho")


def converge(n, bdy, f, omega=None, tol=1e-13, max_iters=200000):
    res = oracle.sor_f64(np.zeros((n, n)), bdy, f,
                         omega_opt(n) if omega is None else omega, tol,
                         max_iters, 1)
    assert res.status == oracle.OK, res
    return res


# ---------------------------------------------------------------------------
# Hand-worked examples and closed forms
# ---------------------------------------------------------------------------

def test_n2_hand_worked_example():
    g = _load("n2_hand.json")
    bdy = np.array(g["boundary"], float)
    for k in ("1", "2"):
        res = oracle.sor_f64(np.array(g["u0"], float), bdy, None, g["omega"],
                             0.0, int(k), 1, hist=True)
        assert res.status == oracle.NOT_CONVERGED
        assert res.iterations == int(k)
        np.testing.assert_array_equal(res.u, np.array(g["after"][k]["u"]))
        assert res.mhist[-1] == g["after"][k]["max_change"]
        assert res.final_max_delta == g["after"][k]["max_change"]


def test_n2_hand_worked_example_float_storage():
    g = _load("n2_hand.json")
    bdy = np.array(g["boundary"], float)
    res = oracle.sor_f32(np.zeros((2, 2)), bdy, None, g["omega"], 0.0, 2, 1)
    np.testing.assert_array_equal(res.u.astype(float), np.array(g["after"]["2"]["u"]))


def test_n1_poisson_hand_worked_example():
    g = _load("n1_poisson_hand.json")
    res = oracle.sor_f64(np.zeros((1, 1)), np.array(g["boundary"], float),
                         np.array(g["f"], float), g["omega"], 0.0, 3, 1, hist=True)
    assert res.u[0, 0] == g["u"][-1]
    np.testing.assert_array_equal(res.mhist, np.array(g["max_change"]))


@pytest.mark.parametrize("omega", [0.376, 1.0, 1.37, 1.9])
def test_n1_closed_form(omega):
    """One red cell: u_k = u*(1 - (1-w)^k), change_k = |u*| w |1-w|^(k-1)."""
    rng = np.random.default_rng(11)
    bdy = rng.uniform(0, 100, 4)
    f = rng.standard_normal((1, 1)) * 50
    ustar = (bdy.sum() + 0.25 * f[0, 0]) / 4.0
    res = oracle.sor_f64(np.zeros((1, 1)), bdy, f, omega, 0.0, 40, 1, hist=True)
    k = np.arange(1, 41)
    expect_change = abs(ustar) * omega * abs(1 - omega) ** (k - 1)
    np.testing.assert_allclose(res.mhist, expect_change, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(res.u[0, 0], ustar * (1 - (1 - omega) ** 40),
                               rtol=1e-13)


def test_n1_stop_iteration_is_first_passing_check():
    """With K = 1 the returned iteration is the first k with change_k < tol."""
    bdy = np.array([40.0, 0.0, 0.0, 0.0])
    omega, tol = 0.5, 1e-3
    ustar = 10.0
    k = 1
    while abs(ustar) * omega * (1 - omega) ** (k - 1) >= tol:
        k += 1
    res = oracle.sor_f64(np.zeros((1, 1)), bdy, None, omega, tol, 1000, 1)
    assert res.status == oracle.OK and res.iterations == k


# ---------------------------------------------------------------------------
# Converged solution against independent solvers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,with_f", [(3, True), (8, False), (17, True), (32, True)])
def test_converged_matches_dense_direct_solve(n, with_f):
    rng = np.random.default_rng(100 + n)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n)) * 100 if with_f else None
    res = converge(n, bdy, f)
    ref = dense_solve(n, bdy, f)
    assert np.max(np.abs(res.u - ref)) <= 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [64, 127])
def test_converged_matches_dst(n):
    rng = np.random.default_rng(200 + n)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n))
    res = converge(n, bdy, f, tol=1e-12)
    ref = dst_solve(n, bdy, f)
    assert np.max(np.abs(res.u - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_dst_matches_dense():
    """The two independent exact solvers agree (pins the DST helper itself)."""
    n = 12
    rng = np.random.default_rng(5)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n))
    np.testing.assert_allclose(dst_solve(n, bdy, f), dense_solve(n, bdy, f),
                               rtol=1e-12, atol=1e-10)


def test_manufactured_solution_second_order():
    """f = 2 pi^2 sin(pi x) sin(pi y), zero boundary: the discrete solution is
    c(h) sin(pi x) sin(pi y), c(h) = (pi h/2)^2 / sin^2(pi h/2), and its error
    against the continuum solution falls by 4 when h halves."""
    errs = []
    for n in (15, 31, 63):
        h = 1.0 / (n + 1)
        f = manufactured_term(n)
        res = converge(n, np.zeros(4 * n), f, tol=1e-14)
        s = np.sin(np.pi * h * np.arange(1, n + 1))
        c = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
        np.testing.assert_allclose(res.u, c * np.outer(s, s), rtol=0, atol=1e-11)
        errs.append(np.max(np.abs(res.u - np.outer(s, s))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.9 < r1 < 4.1 and 3.95 < r2 < 4.05


def test_top_edge_separation_of_variables():
    """Laplace with a top-edge profile g: u_ij = sum_k a_k sin(k pi j h)
    sinh(b_k (n+1-i)) / sinh(b_k (n+1)), cosh b_k = 2 - cos(k pi h)."""
    n = 32
    g = laplace_top_edge(n)
    res = converge(n, g.bdy, None)
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    top = g.bdy[:n]
    ref = np.zeros((n, n))
    for k in range(1, n + 1):
        a = 2.0 / (n + 1) * np.sum(top * np.sin(k * np.pi * j * h))
        beta = math.acosh(2.0 - math.cos(k * np.pi * h))
        i = np.arange(1, n + 1)
        # sinh(b (n+1-i)) / sinh(b (n+1)) in overflow-free form
        ratio = np.exp(-beta * i) * (1 - np.exp(-2 * beta * (n + 1 - i))) / (
            1 - np.exp(-2 * beta * (n + 1)))
        ref += a * np.outer(ratio, np.sin(k * np.pi * j * h))
    np.testing.assert_allclose(res.u, ref, rtol=0, atol=1e-9)


def test_max_principle_and_mirror_symmetry():
    n = 64
    g = laplace_top_edge(n)
    res = converge(n, g.bdy, None, tol=1e-12)
    assert res.u.min() >= 0.0 and res.u.max() <= 100.0
    np.testing.assert_allclose(res.u, res.u[:, ::-1], rtol=0, atol=1e-9)
    rng = np.random.default_rng(3)
    bdy = rng.uniform(20, 60, 4 * n)
    res = converge(n, bdy, None, tol=1e-12)
    assert res.u.min() >= bdy.min() - 1e-9 and res.u.max() <= bdy.max() + 1e-9


def test_iterates_obey_max_principle_for_underrelaxation():
    n = 20
    rng = np.random.default_rng(8)
    bdy = rng.uniform(10, 90, 4 * n)
    for k in (1, 5, 30):
        res = oracle.sor_f64(np.zeros((n, n)), bdy, None, 0.8, 0.0, k, 1)
        assert res.u.min() >= 0.0 and res.u.max() <= bdy.max()


# ---------------------------------------------------------------------------
# Convergence rates (Young's theory; red-black ordering is consistently ordered)
# ---------------------------------------------------------------------------

def _tail_ratio(n, omega, iters, lo=None):
    """Geometric-mean decay ratio of the per-iteration max change over the
    second half of the iterations before the changes reach 1e-9 of the first
    (well above rounding level), or from iteration lo on."""
    rng = np.random.default_rng(1)
    bdy = rng.uniform(0, 100, 4 * n)
    res = oracle.sor_f64(np.zeros((n, n)), bdy, None, omega, 0.0, iters, 1,
                         hist=True)
    m = res.mhist
    hi = int(np.argmax(m < 1e-9 * m[0])) if np.any(m < 1e-9 * m[0]) else len(m)
    lo = hi // 2 if lo is None else lo
    assert hi - lo > 20, (lo, hi)
    m = m[lo:hi]
    return float(np.exp(np.mean(np.log(m[1:] / m[:-1]))))


def test_gauss_seidel_rate_is_jacobi_radius_squared():
    n = 16
    mu = math.cos(math.pi / (n + 1))            # Jacobi spectral radius
    ratio = _tail_ratio(n, 1.0, 700, 150)
    assert abs(ratio - mu * mu) < 2e-4


@pytest.mark.parametrize("omega", [0.376, 1.3, 1.6])
def test_sor_rate_matches_young_root(omega):
    n = 16
    mu = math.cos(math.pi / (n + 1))
    # largest root of (lam + w - 1)^2 = lam w^2 mu^2
    bq = 2 * (omega - 1) - omega ** 2 * mu ** 2
    lam = (-bq + math.sqrt(bq * bq - 4 * (omega - 1) ** 2)) / 2
    iters = 3000 if omega < 1 else 600
    ratio = _tail_ratio(n, omega, iters)
    assert abs(ratio - lam) < 5e-4


def test_overrelaxed_rate_is_omega_minus_one():
    n = 16
    omega = 1.85                                  # above omega_opt(16) = 1.6895
    ratio = _tail_ratio(n, omega, 1200, 60)
    assert abs(ratio - (omega - 1)) < 2e-2


def test_iteration_count_minimised_near_omega_opt():
    n = 32
    rng = np.random.default_rng(2)
    bdy = rng.uniform(0, 100, 4 * n)
    omegas = np.round(np.arange(1.70, 1.951, 0.005), 4)
    counts = []
    for w in omegas:
        res = oracle.sor_f64(np.zeros((n, n)), bdy, None, float(w), 1e-10,
                             100000, 1)
        counts.append(res.iterations)
    best = omegas[int(np.argmin(counts))]
    assert abs(best - omega_opt(n)) <= 0.02, (best, omega_opt(n))


# ---------------------------------------------------------------------------
# Semantics of the stopping rule and of parallel workers
# ---------------------------------------------------------------------------

def test_change_equals_copy_based_difference():
    """Algorithm 1 copies the grid before a checked iteration and compares; the
    max of per-update changes must equal that difference exactly."""
    n = 23
    rng = np.random.default_rng(4)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n))
    w = omega_opt(n)
    for k in (1, 7, 40):
        a = oracle.sor_f64(np.zeros((n, n)), bdy, f, w, 0.0, k, 1)
        b = oracle.sor_f64(np.zeros((n, n)), bdy, f, w, 0.0, k + 1, 1, hist=True)
        assert np.max(np.abs(b.u - a.u)) == b.mhist[-1]


def test_check_cadence_and_strict_comparison():
    n = 20
    rng = np.random.default_rng(6)
    bdy = rng.uniform(0, 100, 4 * n)
    w = omega_opt(n)
    full = oracle.sor_f64(np.zeros((n, n)), bdy, None, w, 0.0, 400, 1, hist=True)
    tol = 1e-6
    res = oracle.sor_f64(np.zeros((n, n)), bdy, None, w, tol, 400, 10)
    first = next(k for k in range(10, 401, 10) if full.mhist[k - 1] < tol)
    assert res.iterations == first and res.final_max_delta == full.mhist[first - 1]
    # strict: a tolerance equal to a checked change does not stop there
    exact = full.mhist[first - 1]
    res2 = oracle.sor_f64(np.zeros((n, n)), bdy, None, w, exact, 400, 10)
    assert res2.iterations > first
    # the last allowed iteration is always checked
    res3 = oracle.sor_f64(np.zeros((n, n)), bdy, None, w, 1e30, 7, 10)
    assert res3.status == oracle.OK and res3.iterations == 7


def test_threaded_workers_bitwise_equal_serial():
    n = 57
    rng = np.random.default_rng(9)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n))
    a = oracle.sor_f64(np.zeros((n, n)), bdy, f, 1.9, 0.0, 60, 1, threads=1, hist=True)
    b = oracle.sor_f64(np.zeros((n, n)), bdy, f, 1.9, 0.0, 60, 1, threads=4, hist=True)
    np.testing.assert_array_equal(a.u, b.u)
    np.testing.assert_array_equal(a.mhist, b.mhist)


def test_invalid_arguments_and_nonfinite():
    bdy = np.ones(8)
    for kw in (dict(omega=0.0), dict(omega=2.0), dict(tol=float("nan")),
               dict(max_iters=0), dict(check_every=0)):
        args = dict(omega=1.0, tol=1e-6, max_iters=10, check_every=1)
        args.update(kw)
        with pytest.raises(ValueError):
            oracle.sor_f64(np.zeros((2, 2)), bdy, None, **args)
    bad = bdy.copy()
    bad[3] = np.nan
    res = oracle.sor_f64(np.zeros((2, 2)), bad, None, 1.0, 1e-6, 10, 1)
    assert res.status == oracle.ENONFINITE


@pytest.mark.parametrize("bits", [32, 16])
def test_mixed_nonfinite_data_never_converges(bits):
    """A NaN in the source or an infinite boundary value has no solution, and
    entries of about 1e200 overflow the 2-norms the stopping rule uses: each
    ends the mixed solve with ENONFINITE before any correction.  (A NaN that
    spreads through the grid drops out of the max |r| comparisons, so max |r|
    alone would read as zero, i.e. as an exact solution.)"""
    n = 9
    rng = np.random.default_rng(5)
    bdy = rng.uniform(0.0, 1.0, 4 * n)
    f = rng.standard_normal((n, n))
    nan_f = f.copy()
    nan_f[4, 2] = np.nan
    inf_b = bdy.copy()
    inf_b[n + 3] = np.inf
    for b, ff in ((bdy, nan_f), (inf_b, f), (bdy * 1e200, None)):
        res = oracle.mixed(np.zeros((n, n)), b, ff, 1.5, 1e-10, 5, bits, 2 * n)
        assert res.status == oracle.ENONFINITE and res.outer_steps == 0
        assert not math.isfinite(res.rel_residual)
    res = oracle.mixed(np.zeros((n, n)), bdy * 1e100, f, 1.5, 1e-10, 40, bits, 4 * n)
    assert res.status == oracle.OK and math.isfinite(res.rel_residual)


# ---------------------------------------------------------------------------
# Residual
# ---------------------------------------------------------------------------

def test_residual_matches_dense_operator():
    n = 14
    rng = np.random.default_rng(12)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n)) * 300
    u = rng.uniform(0, 100, (n, n))
    A, b = dense_system(n, bdy, f)
    r, sr, sb, mr = oracle.residual_f64(u, bdy, f)
    ref = (b - A @ u.ravel()).reshape(n, n)
    np.testing.assert_allclose(r, ref, rtol=0, atol=1e-11)
    np.testing.assert_allclose(sr, np.sum(ref ** 2), rtol=1e-12)
    np.testing.assert_allclose(sb, np.sum(b ** 2), rtol=1e-12)
    np.testing.assert_allclose(mr, np.max(np.abs(ref)), rtol=1e-12)
    ustar = dense_solve(n, bdy, f)
    assert oracle.rel_residual(ustar, bdy, f) < 1e-14


# ---------------------------------------------------------------------------
# Reduced precision
# ---------------------------------------------------------------------------

def test_round_half_matches_numpy_binary16():
    rng = np.random.default_rng(13)
    xs = np.concatenate([
        rng.standard_normal(4000).astype(np.float32) * 10.0,
        (rng.uniform(-1, 1, 2000) * 2.0 ** rng.integers(-30, 17, 2000)).astype(np.float32),
        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, -65520.0, 1e-8, 2.0 ** -24,
                  2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14, 1.0 + 2.0 ** -11,
                  1.0 + 3 * 2.0 ** -11, 2049.0, 2051.0, 4097.0], dtype=np.float32),
    ])
    with np.errstate(over="ignore"):
        ref = xs.astype(np.float16).astype(np.float32)
    got = np.array([oracle.round_half(float(x)) for x in xs], dtype=np.float32)
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_float_storage_converges_to_float_accuracy():
    n = 40
    rng = np.random.default_rng(14)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.standard_normal((n, n)) * 100
    ref = dst_solve(n, bdy, f)
    res = oracle.sor_f32(np.zeros((n, n)), bdy, f, omega_opt(n), 1e-4, 20000, 1)
    assert res.status == oracle.OK
    assert np.max(np.abs(res.u - ref)) < 1e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("bits,tol", [(32, 1e-13), (16, 1e-11)])
def test_mixed_precision_refinement_reaches_fp64_accuracy(bits, tol):
    n = 63
    rng = np.random.default_rng(15)
    f = manufactured_term(n) + rng.standard_normal((n, n))
    bdy = np.zeros(4 * n)
    res = oracle.mixed(np.zeros((n, n)), bdy, f, omega_opt(n), tol, 40, bits, 2 * n)
    assert res.converged, res.relhist
    assert res.rel_residual <= tol
    assert np.all(np.diff(res.relhist) < 0)          # every correction helps
    ref = dst_solve(n, bdy, f)
    assert np.max(np.abs(res.u - ref)) <= 1e-9 * np.max(np.abs(ref))
    # cross-check the returned rel against the residual routine
    assert abs(oracle.rel_residual(res.u, bdy, f) - res.rel_residual) <= 1e-3 * tol


@pytest.mark.parametrize("bits", [32, 16])
def test_mixed_correction_size_stop_rule(bits):
    """The second stopping rule of the mixed solve: after at least one
    correction, stop when the last correction's largest magnitude is below
    corr_tol.  The corrections are measured here from the iterates themselves
    (u_k - u_{k-1}, from runs limited to k and k-1 corrections), not from the
    oracle's own report: the first one exactly (u_0 = 0, so u_1 is the
    correction), later ones to within a rounding of u.  A rule tested before
    the correction is added, or on the scaled correction (without 2^-p), or
    allowed before any correction, fails here."""
    n = 21
    rng = np.random.default_rng(16)
    bdy = rng.uniform(0.0, 100.0, 4 * n)
    f = rng.standard_normal((n, n)) * 50.0
    omega = omega_opt(n)
    inner = 6                      # weak inner solves: corrections shrink slowly
    K = 7
    us = [np.zeros((n, n))]
    for k in range(1, K + 1):
        r = oracle.mixed(np.zeros((n, n)), bdy, f, omega, 0.0, k, bits, inner)
        assert r.outer_steps == k and r.status == oracle.NOT_CONVERGED
        us.append(r.u)
    c = [None] + [float(np.max(np.abs(us[k] - us[k - 1]))) for k in range(1, K + 1)]
    assert all(c[k + 1] < c[k] * 0.9 for k in range(1, K)), c   # strictly shrinking
    run = lambda tol: oracle.mixed(np.zeros((n, n)), bdy, f, omega, 0.0, K + 3, bits,
                                   inner, corr_tol=tol)
    # The first correction is u_1 exactly: its size is the returned one.
    r1 = run(c[1] * (1 + 1e-9))
    assert r1.status == oracle.OK and r1.outer_steps == 1
    assert r1.last_correction == c[1]
    np.testing.assert_array_equal(r1.u, us[1])
    assert run(c[1]).outer_steps == 2           # strict: c_1 < c_1 is false
    # A threshold just above (below) c_j stops after j (j + 1) corrections,
    # returning the iterate that includes the last correction.
    for j in range(2, K):
        hi, lo = run(c[j] * (1 + 1e-6)), run(c[j] * (1 - 1e-6))
        assert hi.status == oracle.OK and hi.outer_steps == j, (j, hi.outer_steps)
        assert lo.status == oracle.OK and lo.outer_steps == j + 1, (j, lo.outer_steps)
        np.testing.assert_array_equal(hi.u, us[j])
        np.testing.assert_array_equal(lo.u, us[j + 1])
        assert abs(hi.last_correction - c[j]) <= 1e-9 * c[j]
    # A huge corr_tol still applies one correction first; max_outer = 0
    # applies none and the rule never fires.
    big = run(1e300)
    assert big.outer_steps == 1 and big.status == oracle.OK
    r0 = oracle.mixed(np.zeros((n, n)), bdy, f, omega, 0.0, 0, bits, inner, corr_tol=1e300)
    assert r0.outer_steps == 0 and r0.status == oracle.NOT_CONVERGED
    # The residual rule is tested first: with rel_tol above the starting
    # residual no correction is applied at all.
    r_rel = oracle.mixed(np.zeros((n, n)), bdy, f, omega, 2.0, K, bits, inner, corr_tol=1e300)
    assert r_rel.outer_steps == 0 and r_rel.status == oracle.OK


def test_mixed_threads_bitwise_equal_serial():
    n = 37
    rng = np.random.default_rng(17)
    bdy = rng.uniform(0.0, 100.0, 4 * n)
    f = rng.standard_normal((n, n))
    for bits in (32, 16):
        a = oracle.mixed(np.zeros((n, n)), bdy, f, omega_opt(n), 0.0, 3, bits, 2 * n)
        b = oracle.mixed(np.zeros((n, n)), bdy, f, omega_opt(n), 0.0, 3, bits, 2 * n,
                         threads=4)
        np.testing.assert_array_equal(a.u.view(np.uint64), b.u.view(np.uint64))
        np.testing.assert_array_equal(a.relhist, b.relhist)
