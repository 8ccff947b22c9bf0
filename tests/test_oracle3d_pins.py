"""Pins of the 3-D oracle (7-point red-black SOR on the unit cube, the 3-D form
of Mittal 2014's method named as future work in Sec. 5) against facts that do
not come from the oracle: the closed form for one cell, a dense direct solve
of the assembled 7-point system, the discrete eigenfunction sin sin sin,
second-order convergence to the continuous solution, Young's convergence
rates (Jacobi radius mu = cos(pi h) for the 7-point stencil), the discrete
maximum principle and the symmetry of the cube."""
import math

import numpy as np
import pytest

import oracle

SIXTH = 1.0 / 6.0


def faces_from_function(n, g):
    """The six boundary faces (x=0, x=n+1 [z][y]; y=0, y=n+1 [z][x];
    z=0, z=n+1 [y][x]) of a function g(z, y, x) of full-array indices."""
    idx = np.arange(1, n + 1)
    A, C = np.meshgrid(idx, idx, indexing="ij")
    return np.stack([g(A, C, 0 * A), g(A, C, 0 * A + n + 1),
                     g(A, 0 * A, C), g(A, 0 * A + n + 1, C),
                     g(0 * A, A, C), g(0 * A + n + 1, A, C)]).astype(np.float64)


def dense_system(n, bdy, f):
    """6u - (interior neighbours) = h^2 f + (boundary neighbours), unknowns
    ordered like the oracle's u ([z][y][x], x fastest)."""
    N = n ** 3
    A = np.zeros((N, N))
    b = np.zeros(N)
    h2 = (1.0 / (n + 1)) ** 2
    full = np.zeros((n + 2,) * 3)
    F = faces = bdy.reshape(6, n, n)
    full[1:-1, 1:-1, 0] = F[0]
    full[1:-1, 1:-1, -1] = F[1]
    full[1:-1, 0, 1:-1] = F[2]
    full[1:-1, -1, 1:-1] = F[3]
    full[0, 1:-1, 1:-1] = F[4]
    full[-1, 1:-1, 1:-1] = F[5]
    del faces

    def k(z, y, x):
        return ((z - 1) * n + (y - 1)) * n + (x - 1)
    for z in range(1, n + 1):
        for y in range(1, n + 1):
            for x in range(1, n + 1):
                r = k(z, y, x)
                A[r, r] = 6.0
                b[r] = h2 * f[z - 1, y - 1, x - 1] if f is not None else 0.0
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                   (0, 0, 1), (0, 0, -1)):
                    zz, yy, xx = z + dz, y + dy, x + dx
                    if 1 <= zz <= n and 1 <= yy <= n and 1 <= xx <= n:
                        A[r, k(zz, yy, xx)] = -1.0
                    else:
                        b[r] += full[zz, yy, xx]
    return A, b


def test_one_cell_closed_form():
    """n = 1: the cell's Gauss-Seidel value g is fixed, so u_k = g (1 - (1-w)^k)
    and the change of iteration k is |g| w |1-w|^(k-1)."""
    bdy = np.array([3.0, -1.5, 2.25, 7.0, 0.5, 4.0])
    g = SIXTH * (((bdy[0] + bdy[1]) + (bdy[2] + bdy[3])) + (bdy[4] + bdy[5]))
    for w in (0.376, 1.0, 1.6):
        r = oracle.sor3d_f64(np.zeros((1, 1, 1)), bdy, None, w, 0.0, 12, 1, hist=True)
        k = np.arange(1, 13)
        np.testing.assert_allclose(r.mhist, abs(g) * w * abs(1 - w) ** (k - 1), rtol=1e-12, atol=1e-300)
        assert r.u[0, 0, 0] == pytest.approx(g * (1 - (1 - w) ** 12), rel=1e-13)


def test_hand_worked_first_iteration_colour_order():
    """n = 2, zero interior, one boundary value 6 on the x = 0 face next to
    cell (1, 1, 1), which is black (1+1+1 odd).  Red half-sweep first: every
    red cell sees only zeros and stays 0.  Black half-sweep: cell (1, 1, 1)
    has s = 6 and g = 6 * fl(1/6) = fl(1 - 2^-54) = 1 (a tie, rounded to even),
    so it becomes 0 + w (1 - 0) = w; the other black cells stay 0.  The change
    of the iteration is w.  (Black first would give the red neighbours of
    (1, 1, 1) the value fl(w/6)-ish instead of 0.)"""
    n, w = 2, 1.5
    bdy = np.zeros((6, n, n))
    bdy[0, 0, 0] = 6.0                   # face x = 0 at (z, y) = (1, 1)
    r = oracle.sor3d_f64(np.zeros((n, n, n)), bdy, None, w, 0.0, 1, 1, hist=True)
    expect = np.zeros((n, n, n))
    expect[0, 0, 0] = w
    assert np.array_equal(r.u, expect)
    assert r.mhist[0] == w


@pytest.mark.parametrize("n", [2, 3, 5])
def test_converged_solution_matches_dense_solve(n):
    rng = np.random.default_rng(100 + n)
    bdy = rng.uniform(0, 100, size=(6, n, n))
    f = rng.standard_normal((n, n, n)) * 50
    A, b = dense_system(n, bdy, f)
    ref = np.linalg.solve(A, b).reshape(n, n, n)
    w = 2.0 / (1.0 + math.sin(math.pi / (n + 1)))
    # tol 1e-13: boundary values up to 100 have an ulp of 1.4e-14, so a
    # smaller change would require an exact fixed point of the rounded update
    r = oracle.sor3d_f64(np.zeros((n, n, n)), bdy, f, w, 1e-13, 100000, 1)
    assert r.status == oracle.OK
    np.testing.assert_allclose(r.u, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_manufactured_eigenfunction_and_second_order():
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), zero boundary: the discrete
    solution is (3 pi^2 / lam_h) sin sin sin with lam_h = (12/h^2) sin^2(pi h/2),
    and its error against the continuous solution falls 4x when h halves."""
    errs = []
    for n in (7, 15):
        h = 1.0 / (n + 1)
        s = np.sin(np.pi * h * np.arange(1, n + 1))
        mode = s[:, None, None] * s[None, :, None] * s[None, None, :]
        f = 3 * np.pi ** 2 * mode
        lam = 12.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2
        w = 2.0 / (1.0 + math.sin(math.pi * h))
        r = oracle.sor3d_f64(np.zeros((n, n, n)), np.zeros((6, n, n)), f, w, 1e-15, 200000, 1)
        assert r.status == oracle.OK
        np.testing.assert_allclose(r.u, 3 * np.pi ** 2 / lam * mode, rtol=0, atol=1e-12)
        errs.append(np.abs(r.u - mode).max())
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.02)


def _late_ratio(mh):
    return mh[-1] / mh[-2]


@pytest.mark.parametrize("n", [9, 15])
def test_young_rates(n):
    """mu = cos(pi h) for the 7-point Jacobi matrix.  Gauss-Seidel (w = 1)
    decays as mu^2; for w below the optimum the rate is the largest root of
    (l + w - 1)^2 = l w^2 mu^2; above it, |l| = w - 1."""
    h = 1.0 / (n + 1)
    mu = math.cos(math.pi * h)
    rng = np.random.default_rng(n)
    bdy = rng.uniform(0, 1, size=(6, n, n))
    u0 = rng.uniform(0, 1, size=(n, n, n))
    def iters(rate):      # long enough to be asymptotic, short of rounding
        return int(math.log(1e-9) / math.log(rate))
    r = oracle.sor3d_f64(u0, bdy, None, 1.0, 0.0, iters(mu ** 2), 1, hist=True)
    assert _late_ratio(r.mhist) == pytest.approx(mu ** 2, rel=2e-3)
    w = 1.3
    c = w * w * mu * mu
    # (l + w - 1)^2 = l c  ->  l^2 + (2(w-1) - c) l + (w-1)^2 = 0
    bq = 2 * (w - 1) - c
    lam = (-bq + math.sqrt(bq * bq - 4 * (w - 1) ** 2)) / 2
    r = oracle.sor3d_f64(u0, bdy, None, w, 0.0, iters(lam), 1, hist=True)
    assert _late_ratio(r.mhist) == pytest.approx(lam, rel=2e-3)
    w = 1.85
    r = oracle.sor3d_f64(u0, bdy, None, w, 0.0, iters(w - 1), 1, hist=True)
    mh = r.mhist[-60:]
    rate = (mh[-1] / mh[0]) ** (1.0 / (len(mh) - 1))
    assert rate == pytest.approx(w - 1, rel=0.02)


def test_maximum_principle_and_cube_symmetry():
    n = 6
    rng = np.random.default_rng(7)
    # Boundary data of a function, so the face values agree where faces meet
    # only through the function itself (edges and corners are never read).
    B = rng.uniform(0, 100, size=(n + 2, n + 2, n + 2))
    bdy = faces_from_function(n, lambda z, y, x: B[z, y, x])
    w = 2.0 / (1.0 + math.sin(math.pi / (n + 1)))
    r = oracle.sor3d_f64(np.zeros((n, n, n)), bdy, None, w, 1e-12, 100000, 1)
    assert r.status == oracle.OK
    assert r.u.min() >= bdy.min() - 1e-12 and r.u.max() <= bdy.max() + 1e-12
    # Swap the x and y axes of the boundary function: the solution transposes
    # (up to rounding, since the sum order is not symmetric).
    Bt = np.swapaxes(B, 1, 2)
    bdy_t = faces_from_function(n, lambda z, y, x: Bt[z, y, x])
    rt = oracle.sor3d_f64(np.zeros((n, n, n)), bdy_t, None, w, 1e-12, 100000, 1)
    np.testing.assert_allclose(np.swapaxes(rt.u, 1, 2), r.u, rtol=0, atol=1e-10)


def test_threads_bitwise_and_cadence():
    n = 12
    rng = np.random.default_rng(3)
    bdy = rng.uniform(0, 100, size=(6, n, n))
    f = rng.standard_normal((n, n, n))
    a = oracle.sor3d_f64(np.zeros((n, n, n)), bdy, f, 1.7, 1e-6, 500, 7, threads=1, hist=True)
    b = oracle.sor3d_f64(np.zeros((n, n, n)), bdy, f, 1.7, 1e-6, 500, 7, threads=4, hist=True)
    assert np.array_equal(a.u.view(np.uint64), b.u.view(np.uint64))
    assert a.iterations == b.iterations and a.iterations % 7 == 0
    assert np.array_equal(a.mhist, b.mhist)
    # the check passed at the first multiple of 7 whose change is < tol
    k = a.iterations
    assert a.mhist[k - 1] < 1e-6 and all(a.mhist[j - 1] >= 1e-6 for j in range(7, k, 7))
