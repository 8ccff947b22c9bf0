"""Pins of the oracle's Jacobi and four-colour orderings (the alternatives to
red-black that Mittal 2014 names: Jacobi in Sec. 2.1, multi-colour SOR in
Sec. 3.1) against facts that do not come from the oracle: hand-worked first
iterations that fix each order, the one-cell closed form, the discrete
solution (dense solve and the DST diagonalisation), Jacobi's spectral radius
cos(pi h) and the over-relaxed Jacobi rate, Young's rates (the four-colour
order is consistently ordered, so it obeys the red-black relation between
omega and the rate), exact transpose symmetry and the maximum principle."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_pins import dense_solve, dst_solve
from workloads import omega_opt

J, C4 = oracle.ORDER_JACOBI, oracle.ORDER_FOUR_COLOUR


def south_only(n, j, value):
    """Boundary (N, S, W, E) that is 0 except the south edge at column j."""
    b = np.zeros(4 * n)
    b[n + j - 1] = value
    return b


def test_four_colour_hand_worked_first_iteration():
    """n = 2, zero interior, south boundary 4 below cell (2, 2).  Colours of
    the full array: (2,2) -> 0, (2,1) -> 1, (1,2) -> 2, (1,1) -> 3.  With
    w = 1: (2,2) = 4/4 = 1; (2,1) and (1,2) each see it: 1/4; (1,1) sees
    both: (1/4 + 1/4)/4 = 1/8.  With w = 1.5: 1.5, 1.5*(1.5/4) = 0.5625
    twice, 1.5*(1.125/4) = 0.421875.  Red-black would leave (1,1) at 0 (it is
    red and updated first) and reversed colours would leave (2,1), (1,2) at
    0; all values are exact in binary."""
    b = south_only(2, 2, 4.0)
    r = oracle.variant_f64(C4, np.zeros((2, 2)), b, None, 1.0, 0.0, 1, 1, hist=True)
    np.testing.assert_array_equal(r.u, [[0.125, 0.25], [0.25, 1.0]])
    assert r.mhist[0] == 1.0
    r = oracle.variant_f64(C4, np.zeros((2, 2)), b, None, 1.5, 0.0, 1, 1, hist=True)
    np.testing.assert_array_equal(r.u, [[0.421875, 0.5625], [0.5625, 1.5]])
    rb = oracle.sor_f64(np.zeros((2, 2)), b, None, 1.0, 0.0, 1, 1)
    np.testing.assert_array_equal(rb.u, [[0.0, 0.25], [0.25, 1.0]])


def test_jacobi_hand_worked_two_iterations():
    """Same set-up: Jacobi reads only the previous iterate, so iteration 1
    changes only (2, 2) (to 1) and iteration 2 gives (2,1) = (1,2) = 1/4 with
    (1,1) still 0; the changes are 1 and 1/4."""
    b = south_only(2, 2, 4.0)
    r = oracle.variant_f64(J, np.zeros((2, 2)), b, None, 1.0, 0.0, 1, 1, hist=True)
    np.testing.assert_array_equal(r.u, [[0.0, 0.0], [0.0, 1.0]])
    r = oracle.variant_f64(J, np.zeros((2, 2)), b, None, 1.0, 0.0, 2, 1, hist=True)
    np.testing.assert_array_equal(r.u, [[0.0, 0.25], [0.25, 1.0]])
    np.testing.assert_array_equal(r.mhist, [1.0, 0.25])


@pytest.mark.parametrize("ordering", [J, C4])
def test_one_cell_closed_form(ordering):
    b = np.array([3.0, -1.0, 2.5, 7.5])
    g = 0.25 * ((b[0] + b[1]) + (b[2] + b[3]))
    for w in (0.376, 1.0, 1.7):
        r = oracle.variant_f64(ordering, np.zeros((1, 1)), b, None, w, 0.0, 10, 1, hist=True)
        k = np.arange(1, 11)
        np.testing.assert_allclose(r.mhist, abs(g) * w * abs(1 - w) ** (k - 1), rtol=1e-12)
        assert r.u[0, 0] == pytest.approx(g * (1 - (1 - w) ** 10), rel=1e-13)


@pytest.mark.parametrize("ordering,n", [(J, 6), (J, 9), (C4, 7), (C4, 16)])
def test_converged_solution_is_the_discrete_solution(ordering, n):
    rng = np.random.default_rng(40 + n)
    b = rng.uniform(0, 100, size=4 * n)
    f = rng.standard_normal((n, n)) * 100
    w = 1.0 if ordering == J else omega_opt(n)
    r = oracle.variant_f64(ordering, np.zeros((n, n)), b, f, w, 1e-12, 500000, 1)
    assert r.status == oracle.OK
    ref = dense_solve(n, b, f)
    np.testing.assert_allclose(r.u, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(r.u, dst_solve(n, b, f), rtol=0, atol=1e-11 * np.abs(ref).max())


def _rate(mh, window=40):
    tail = np.asarray(mh[-window - 1:])
    return (tail[-1] / tail[0]) ** (1.0 / window)


@pytest.mark.parametrize("n", [9, 15])
def test_jacobi_rates(n):
    """The Jacobi matrix of the 5-point stencil has eigenvalues
    (cos(p pi h) + cos(q pi h))/2, largest magnitude mu = cos(pi h); over-
    relaxed Jacobi with w < 1 has rate 1 - w + w mu."""
    h = 1.0 / (n + 1)
    mu = math.cos(math.pi * h)
    rng = np.random.default_rng(n)
    b = rng.uniform(0, 1, size=4 * n)
    u0 = rng.uniform(0, 1, size=(n, n))
    for w, rate in ((1.0, mu), (0.7, 1 - 0.7 + 0.7 * mu)):
        iters = int(math.log(1e-9) / math.log(rate))
        r = oracle.variant_f64(J, u0, b, None, w, 0.0, iters, 1, hist=True)
        assert _rate(r.mhist) == pytest.approx(rate, rel=2e-3)


@pytest.mark.parametrize("n", [9, 15])
def test_four_colour_young_rates(n):
    """The four-colour order is consistently ordered (levels (0,0) -> 0,
    (0,1) and (1,0) -> 1, (1,1) -> 2 over (i mod 2, j mod 2)), so its rate
    obeys (l + w - 1)^2 = l w^2 mu^2 like red-black: Gauss-Seidel mu^2, below
    the optimum the largest root, above it w - 1."""
    h = 1.0 / (n + 1)
    mu = math.cos(math.pi * h)
    rng = np.random.default_rng(100 + n)
    b = rng.uniform(0, 1, size=4 * n)
    u0 = rng.uniform(0, 1, size=(n, n))
    w = 1.3
    c = w * w * mu * mu
    bq = 2 * (w - 1) - c
    lam = (-bq + math.sqrt(bq * bq - 4 * (w - 1) ** 2)) / 2
    for w_, rate in ((1.0, mu * mu), (1.3, lam)):
        iters = int(math.log(1e-9) / math.log(rate))
        r = oracle.variant_f64(C4, u0, b, None, w_, 0.0, iters, 1, hist=True)
        assert _rate(r.mhist) == pytest.approx(rate, rel=2e-3)
    w = 1.9
    r = oracle.variant_f64(C4, u0, b, None, w, 0.0, 300, 1, hist=True)
    assert _rate(r.mhist, 100) == pytest.approx(w - 1, rel=0.02)


@pytest.mark.parametrize("ordering", [J, C4])
def test_transpose_symmetry_is_exact(ordering):
    """Transposing the problem (u0, f transposed; north <-> west, south <->
    east) transposes every iterate bit for bit: the sum (N+S)+(W+E) only
    swaps its two halves (IEEE addition commutes), and transposition maps
    colours 1 <-> 2, which never touch each other (both border only colours
    0 and 3), so updating 1 then 2 equals updating 2 then 1."""
    n = 11
    rng = np.random.default_rng(5)
    b = rng.uniform(0, 100, size=4 * n)
    f = rng.standard_normal((n, n))
    u0 = rng.uniform(0, 100, size=(n, n))
    bt = np.concatenate([b[2 * n:3 * n], b[3 * n:], b[:n], b[n:2 * n]])
    a = oracle.variant_f64(ordering, u0, b, f, 1.3, 0.0, 37, 1, hist=True)
    t = oracle.variant_f64(ordering, u0.T, bt, f.T, 1.3, 0.0, 37, 1, hist=True)
    assert np.array_equal(a.u.T.view(np.uint64), t.u.view(np.uint64))
    assert np.array_equal(a.mhist, t.mhist)


@pytest.mark.parametrize("ordering", [J, C4])
def test_maximum_principle_and_stop_rule(ordering):
    n = 12
    rng = np.random.default_rng(8)
    b = rng.uniform(10, 90, size=4 * n)
    w = 1.0 if ordering == J else omega_opt(n)
    full = oracle.variant_f64(ordering, np.zeros((n, n)) + 50, b, None, w, 0.0, 2000, 1, hist=True)
    r = oracle.variant_f64(ordering, np.zeros((n, n)) + 50, b, None, w, 1e-6, 2000, 7)
    k = r.iterations
    assert r.status == oracle.OK and k % 7 == 0
    assert full.mhist[k - 1] < 1e-6 and all(full.mhist[j - 1] >= 1e-6 for j in range(7, k, 7))
    assert r.u.min() >= b.min() - 1e-9 and r.u.max() <= b.max() + 1e-9


def test_orderings_differ_and_reject_unknown():
    n = 8
    rng = np.random.default_rng(2)
    b = rng.uniform(0, 100, size=4 * n)
    rb = oracle.sor_f64(np.zeros((n, n)), b, None, 1.4, 0.0, 3, 1)
    a = oracle.variant_f64(J, np.zeros((n, n)), b, None, 1.4, 0.0, 3, 1)
    c = oracle.variant_f64(C4, np.zeros((n, n)), b, None, 1.4, 0.0, 3, 1)
    assert not np.array_equal(rb.u, a.u) and not np.array_equal(rb.u, c.u)
    assert not np.array_equal(a.u, c.u)
    with pytest.raises(ValueError):
        oracle.variant_f64(3, np.zeros((n, n)), b, None, 1.0, 0.0, 3, 1)
