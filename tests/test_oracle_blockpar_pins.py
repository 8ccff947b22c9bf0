"""Pins of the oracle's block-parallel SOR (the third parallel SOR form that
Mittal 2014 names in Sec. 3.1, there with a citation only) against facts that
do not come from the oracle's stencil code: hand-worked iterations on a 2 x 2
grid cut into two blocks, the affine map of one iteration assembled as
matrices from the reading (blocks updated together, red-black inside a block,
a neighbour in another block taken at the previous iterate), its spectral
radius as the asymptotic rate, the two limits (one block is red-black SOR,
one-cell blocks are over-relaxed Jacobi), exact transpose symmetry, where
one iteration may differ from red-black at all, and the discrete solution
as the fixed point."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_pins import dense_solve, dense_system

# 2 x 2 grid: a = (1,1) red, b = (1,2) black, c = (2,1) black, d = (2,2) red.
# Boundary order N1 N2 S1 S2 W1 W2 E1 E2.
HAND_BDY = np.array([4.0, 16.0, 8.0, 12.0, 8.0, 0.0, 0.0, 4.0])


def test_hand_worked_row_blocks():
    """Blocks of one row ({a, b} and {c, d}), w = 1, zero start.
    Iteration 1: red a = ((N1 + c) + (W1 + b))/4 = (4 + 8)/4 = 3 and
    d = ((b + S2) + (c + E2))/4 = (12 + 4)/4 = 4.  Black b sees a in its own
    block (new, 3) but d in the other (old, 0): ((16 + 0) + (3 + 0))/4 = 4.75;
    c sees d in its block (new, 4) and a across the edge (old, 0):
    ((0 + 8) + (0 + 4))/4 = 3.  Red-black would give b = 5.75, c = 3.75.
    Iteration 2 from (3, 4.75, 3, 4): a = ((4 + 3) + (8 + 4.75))/4 = 4.9375,
    d = ((4.75 + 12) + (3 + 4))/4 = 5.9375, b = ((16 + 4) + (4.9375 + 0))/4
    = 6.234375, c = ((3 + 8) + (0 + 5.9375))/4 = 4.234375.  Changes 4.75 and
    1.9375.  All values are exact in binary."""
    r = oracle.blockpar_f64(np.zeros((2, 2)), HAND_BDY, None, 1.0, 1, 2, 0.0, 1, 1)
    np.testing.assert_array_equal(r.u, [[3.0, 4.75], [3.0, 4.0]])
    r = oracle.blockpar_f64(np.zeros((2, 2)), HAND_BDY, None, 1.0, 1, 2, 0.0, 2, 1, hist=True)
    np.testing.assert_array_equal(r.u, [[4.9375, 6.234375], [4.234375, 5.9375]])
    np.testing.assert_array_equal(r.mhist, [4.75, 1.9375])
    rb = oracle.sor_f64(np.zeros((2, 2)), HAND_BDY, None, 1.0, 0.0, 1, 1)
    np.testing.assert_array_equal(rb.u, [[3.0, 5.75], [3.75, 4.0]])


def test_hand_worked_row_blocks_overrelaxed():
    """Same blocks, w = 1.5, one iteration: a = 1.5 * 3 = 4.5, d = 1.5 * 4 = 6,
    b = 1.5 * ((16 + 0) + (4.5 + 0))/4 = 7.6875, c = 1.5 * ((0 + 8) + (0 + 6))/4
    = 5.25."""
    r = oracle.blockpar_f64(np.zeros((2, 2)), HAND_BDY, None, 1.5, 1, 2, 0.0, 1, 1)
    np.testing.assert_array_equal(r.u, [[4.5, 7.6875], [5.25, 6.0]])


def test_hand_worked_column_blocks():
    """Blocks of one column ({a, c} and {b, d}), w = 1, zero start: the red
    values are as above (3, 4); b sees d in its block (new, 4) and a across
    (old, 0): ((16 + 4) + (0 + 0))/4 = 5; c sees a in its block (new, 3) and
    d across (old, 0): ((3 + 8) + (0 + 0))/4 = 2.75."""
    r = oracle.blockpar_f64(np.zeros((2, 2)), HAND_BDY, None, 1.0, 2, 1, 0.0, 1, 1)
    np.testing.assert_array_equal(r.u, [[3.0, 5.0], [2.75, 4.0]])


def affine_map(n, bdy, f, omega, br, bc):
    """M, c with u_next = M u + c for one block-parallel iteration, from the
    splitting: R = I + w P_red (N/4 - I) (the red half-sweep reads only the
    previous iterate), then the black half-sweep with the neighbour matrix
    split into N_in (pairs in one block) and N_out (pairs across blocks):
    u'' = (I + w P_blk (N_in/4 - I)) u' + (w/4) P_blk N_out u + (w/4) P_blk b."""
    A, b = dense_system(n, bdy, f)
    N = 4.0 * np.eye(n * n) - A             # neighbour (adjacency) matrix
    ii, jj = np.divmod(np.arange(n * n), n)  # 0-based interior row, column
    red = ((ii + 1) + (jj + 1)) % 2 == 0
    same = ((ii[:, None] // br) == (ii[None, :] // br)) & \
           ((jj[:, None] // bc) == (jj[None, :] // bc))
    N_in = np.where(same, N, 0.0)
    N_out = N - N_in
    I = np.eye(n * n)
    PR, PB = np.diag(red.astype(float)), np.diag((~red).astype(float))
    R = I + omega * PR @ (N / 4.0 - I)
    cR = omega / 4.0 * PR @ b
    Bm = I + omega * PB @ (N_in / 4.0 - I)
    M = Bm @ R + omega / 4.0 * PB @ N_out
    c = Bm @ cR + omega / 4.0 * PB @ b
    return M, c


@pytest.mark.parametrize("br,bc,omega", [(3, 2, 1.3), (2, 5, 0.8), (1, 1, 1.0), (7, 7, 1.6),
                                         (4, 1, 1.9)])
def test_matches_assembled_affine_map(br, bc, omega):
    """Five iterations on n = 7 (ragged blocks) from a random start, Poisson
    source and random boundary, equal the assembled map to rounding."""
    n = 7
    rng = np.random.default_rng(11)
    u0 = rng.uniform(-1, 1, (n, n))
    bdy = rng.uniform(-2, 2, 4 * n)
    f = rng.normal(size=(n, n)) * 40.0
    M, c = affine_map(n, bdy, f, omega, br, bc)
    u = u0.reshape(-1).copy()
    for k in range(1, 6):
        u = M @ u + c
        r = oracle.blockpar_f64(u0, bdy, f, omega, br, bc, 0.0, k, 1)
        np.testing.assert_allclose(r.u.reshape(-1), u, rtol=0, atol=1e-13 * max(1, np.abs(u).max()))


def test_one_block_is_red_black():
    """A block of at least n x n cells: bit for bit red-black SOR."""
    rng = np.random.default_rng(3)
    for n, (br, bc) in ((9, (9, 9)), (10, (64, 11)), (1, (1, 1))):
        u0 = rng.uniform(-1, 1, (n, n))
        bdy = rng.uniform(0, 100, 4 * n)
        f = rng.normal(size=(n, n))
        for ff in (None, f):
            a = oracle.blockpar_f64(u0, bdy, ff, 1.7, br, bc, 0.0, 40, 1, hist=True)
            b = oracle.sor_f64(u0, bdy, ff, 1.7, 0.0, 40, 1, hist=True)
            assert np.array_equal(a.u.view(np.uint64), b.u.view(np.uint64))
            assert np.array_equal(a.mhist, b.mhist)


def test_one_cell_blocks_are_jacobi():
    """Blocks of one cell: every neighbour is in another block, so every cell
    reads the previous iterate: bit for bit the over-relaxed Jacobi
    iteration."""
    rng = np.random.default_rng(4)
    n = 11
    u0 = rng.uniform(-1, 1, (n, n))
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.normal(size=(n, n))
    for omega in (1.0, 0.7):
        a = oracle.blockpar_f64(u0, bdy, f, omega, 1, 1, 0.0, 30, 1, hist=True)
        b = oracle.variant_f64(oracle.ORDER_JACOBI, u0, bdy, f, omega, 0.0, 30, 1, hist=True)
        assert np.array_equal(a.u.view(np.uint64), b.u.view(np.uint64))
        assert np.array_equal(a.mhist, b.mhist)


def test_one_iteration_differs_from_red_black_only_at_block_edges():
    """From the same start, one iteration can differ from red-black only at
    black cells with a neighbour in another block, and does differ there for
    a generic start."""
    n, br, bc = 13, 4, 3
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-1, 1, (n, n))
    bdy = rng.uniform(0, 100, 4 * n)
    a = oracle.blockpar_f64(u0, bdy, None, 1.4, br, bc, 0.0, 1, 1).u
    b = oracle.sor_f64(u0, bdy, None, 1.4, 0.0, 1, 1).u
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    black = (ii + jj) % 2 == 1
    edge = np.zeros((n, n), bool)
    edge[1:, :] |= (ii[1:, :] // br) != (ii[:-1, :] // br)     # north neighbour across
    edge[:-1, :] |= (ii[:-1, :] // br) != (ii[1:, :] // br)    # south
    edge[:, 1:] |= (jj[:, 1:] // bc) != (jj[:, :-1] // bc)     # west
    edge[:, :-1] |= (jj[:, :-1] // bc) != (jj[:, 1:] // bc)    # east
    differs = a != b
    assert not np.any(differs & ~(black & edge))
    assert np.all(differs[black & edge])


def test_transpose_symmetry():
    """Transposing the problem (north <-> west, south <-> east) and the block
    shape transposes the iterates bit for bit (the sum (N+S)+(W+E) only
    swaps its two halves)."""
    n = 10
    rng = np.random.default_rng(6)
    u0 = rng.uniform(-1, 1, (n, n))
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.normal(size=(n, n))
    bt = np.concatenate([bdy[2 * n:3 * n], bdy[3 * n:4 * n], bdy[0:n], bdy[n:2 * n]])
    a = oracle.blockpar_f64(u0, bdy, f, 1.5, 3, 4, 0.0, 25, 1)
    b = oracle.blockpar_f64(u0.T, bt, f.T, 1.5, 4, 3, 0.0, 25, 1)
    assert np.array_equal(a.u.T.view(np.uint64), np.ascontiguousarray(b.u).view(np.uint64))


@pytest.mark.parametrize("br,bc", [(4, 4), (16, 2), (3, 5)])
def test_rate_is_spectral_radius(br, bc):
    """w = 1 on n = 16 from a random start with zero boundary (solution 0):
    the ratio of successive maximum changes tends to the spectral radius of
    the assembled map, which lies between red-black's cos^2(pi h) and
    Jacobi's cos(pi h)."""
    n = 16
    h = 1.0 / (n + 1)
    M, _ = affine_map(n, np.zeros(4 * n), None, 1.0, br, bc)
    ev = np.linalg.eigvals(M)
    k = np.argsort(-np.abs(ev))
    lam1, lam2 = ev[k[0]], ev[k[1]]
    assert abs(lam1.imag) < 1e-12 and lam1.real > 0 and abs(lam2) < 0.99 * abs(lam1)
    rho = lam1.real
    assert math.cos(math.pi * h) ** 2 < rho < math.cos(math.pi * h)
    rng = np.random.default_rng(7)
    r = oracle.blockpar_f64(rng.uniform(0, 1, (n, n)), np.zeros(4 * n), None, 1.0, br, bc,
                            0.0, 1500, 1, hist=True)
    ratio = r.mhist[1499] / r.mhist[1498]
    assert abs(ratio - rho) < 1e-6 * rho, (ratio, rho)


def test_fixed_point_is_discrete_solution():
    """Iterated to a change below 1e-14, the result is the dense solve's."""
    n = 12
    rng = np.random.default_rng(8)
    bdy = rng.uniform(0, 100, 4 * n)
    f = rng.normal(size=(n, n)) * 50
    r = oracle.blockpar_f64(np.zeros((n, n)), bdy, f, 1.2, 5, 3, 1e-14, 100000, 1)
    assert r.status == oracle.OK
    np.testing.assert_allclose(r.u, dense_solve(n, bdy, f), rtol=0, atol=1e-11)


def test_growth_beyond_the_convergent_range_follows_spectral_radius():
    """Taking the other blocks' old values breaks the consistent ordering
    that lets red-black SOR converge for every w in (0, 2): on n = 12 with
    5 x 3 blocks the assembled map's spectral radius passes 1 between
    w = 1.35 (0.925) and 1.5 (1.122; red-black's is 0.81 there).  The
    oracle's changes follow it: they decay at w = 1.35 and grow by the
    factor |lambda_1| per iteration (over iterations 400..600) at w = 1.5."""
    n, br, bc = 12, 5, 3
    rho = {w: max(abs(np.linalg.eigvals(affine_map(n, np.zeros(4 * n), None, w, br, bc)[0])))
           for w in (1.35, 1.5)}
    assert rho[1.35] < 0.93 and rho[1.5] > 1.12
    assert max(abs(np.linalg.eigvals(affine_map(n, np.zeros(4 * n), None, 1.5, n, n)[0]))) < 0.82
    rng = np.random.default_rng(7)
    u0 = rng.uniform(0, 1, (n, n))
    r = oracle.blockpar_f64(u0, np.zeros(4 * n), None, 1.35, br, bc, 0.0, 600, 1, hist=True)
    assert r.mhist[599] < 1e-15 * r.mhist[0]
    r = oracle.blockpar_f64(u0, np.zeros(4 * n), None, 1.5, br, bc, 0.0, 600, 1, hist=True)
    rate = (r.mhist[599] / r.mhist[399]) ** (1.0 / 200)
    assert abs(rate - rho[1.5]) < 1e-5 * rho[1.5], (rate, rho[1.5])


def test_rejects_bad_block_shape():
    for br, bc in ((0, 1), (1, 0), (-2, 3)):
        with pytest.raises(ValueError):
            oracle.blockpar_f64(np.zeros((3, 3)), np.zeros(12), None, 1.0, br, bc, 0.0, 1, 1)
