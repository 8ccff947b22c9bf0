"""Parity at the largest sides the entry points accept (2-D n = 65536, two
34 GB working grids; 3-D n = 1024) on sampled windows.  After k iterations a
cell depends only on cells within 2k of it (one cell per half-sweep), so the
oracle run on a small window whose ring is frozen at the initial values gives
the exact result more than 2k cells inside that ring; those cells of the GPU
result must agree bit for bit.  Windows sit at the grid's corners, edges and
middle (the ring is then partly the real boundary); each window's offset
keeps the colour parity of its cells."""
import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K_ITERS = 2
R = 8                       # window: interior 2R-1 cells per axis
CORE = slice(2 * K_ITERS + 1, 2 * R - 1 - (2 * K_ITERS + 1))   # cells exact after k


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sor():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1401_0763_amd as m
    return m


def full_value_2d(u0_win_fn, bdy, n):
    """Value of full-array cell (i, j) before the first iteration."""
    def val(i, j):
        if i == 0:
            return bdy[j - 1]
        if i == n + 1:
            return bdy[n + j - 1]
        if j == 0:
            return bdy[2 * n + i - 1]
        if j == n + 1:
            return bdy[3 * n + i - 1]
        return u0_win_fn(i, j)
    return val


def test_2d_largest_side_sampled_windows(sor):
    n = 65536
    ctx = sor.Context(0)
    try:
        rng = np.random.default_rng(65536)
        bdy = rng.uniform(0.0, 100.0, size=4 * n)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(17)
        _say("2-D n=65536: filling u0 on the device")
        u = torch.rand((n, n), dtype=torch.float64, device="cuda", generator=gen) * 100.0
        m = 2 * R - 1
        # window top-left ring corners (full-array indices), even sums
        corners = [(0, 0), (0, n + 1 - 2 * R - 1), (n + 1 - 2 * R - 1, 0),
                   (n + 1 - 2 * R - 1, n + 1 - 2 * R - 1), (n // 2, n // 2 + 2),
                   (1000, 0), (0, 31000), (40002, 2)]
        corners = [(a, b if (a + b) % 2 == 0 else b + 1) for a, b in corners]
        before = {}
        for a, b in corners:
            lo_i, lo_j = max(a - 1, 0), max(b - 1, 0)
            before[(a, b)] = u[lo_i:a + 2 * R, lo_j:b + 2 * R].cpu().numpy().copy()
        omega = 2.0 / (1.0 + np.sin(np.pi / (n + 1)))
        _say("2-D n=65536: solving")
        res = sor.solve_f64(u, torch.tensor(bdy, dtype=torch.float64, device="cuda"), None,
                            omega, 0.0, K_ITERS, 1, hist=False, ctx=ctx)
        assert res.status == sor.NOT_CONVERGED and res.iterations == K_ITERS
        for a, b in corners:
            _say(f"2-D window at ({a}, {b})")
            blk = before[(a, b)]
            lo_i, lo_j = max(a - 1, 0), max(b - 1, 0)
            val = full_value_2d(lambda i, j: blk[i - 1 - lo_i, j - 1 - lo_j], bdy, n)
            w0 = np.array([[val(a + 1 + r, b + 1 + c) for c in range(m)] for r in range(m)])
            wb = np.concatenate([[val(a, b + 1 + c) for c in range(m)],
                                 [val(a + 2 * R, b + 1 + c) for c in range(m)],
                                 [val(a + 1 + r, b) for r in range(m)],
                                 [val(a + 1 + r, b + 2 * R) for r in range(m)]])
            ref = oracle.sor_f64(w0, wb, None, omega, 0.0, K_ITERS, 1)
            got = u[a:a + m, b:b + m].cpu().numpy()          # full (a+1.., b+1..)
            assert np.array_equal(got[CORE, CORE].view(np.uint64),
                                  ref.u[CORE, CORE].view(np.uint64)), (a, b)
        del u
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def test_3d_largest_side_sampled_windows(sor):
    n = 1024
    ctx = sor.Context(0)
    try:
        rng = np.random.default_rng(1024)
        faces = rng.uniform(0.0, 100.0, size=(6, n, n))
        gen = torch.Generator(device="cuda")
        gen.manual_seed(18)
        u = torch.rand((n, n, n), dtype=torch.float64, device="cuda", generator=gen) * 100.0
        m = 2 * R - 1
        corners = [(0, 0, 0), (n + 1 - 2 * R - 1, 0, 0), (0, n + 1 - 2 * R - 1, 2),
                   (n + 1 - 2 * R - 1, n + 1 - 2 * R - 1, n + 1 - 2 * R - 1),
                   (512, 300, 700), (3, 1000, 5)]
        corners = [(a, b, c if (a + b + c) % 2 == 0 else c + 1) for a, b, c in corners]
        before = {}
        for a, b, c in corners:
            lz, ly, lx = max(a - 1, 0), max(b - 1, 0), max(c - 1, 0)
            before[(a, b, c)] = (lz, ly, lx, u[lz:a + 2 * R, ly:b + 2 * R,
                                               lx:c + 2 * R].cpu().numpy().copy())
        omega = 2.0 / (1.0 + np.sin(np.pi / (n + 1)))
        for K in (1, 2):               # one, then two iterations per launch
            _say(f"3-D n=1024 K={K}: solving")
            uu = u.clone()
            res = sor.solve3d_f64(uu, torch.tensor(faces, dtype=torch.float64, device="cuda"),
                                  None, omega, 0.0, K_ITERS, K, ctx=ctx)
            assert res.status == sor.NOT_CONVERGED and res.iterations == K_ITERS
            for a, b, c in corners:
                lz, ly, lx, blk = before[(a, b, c)]

                def val(z, y, x):
                    if x == 0:
                        return faces[0][z - 1][y - 1]
                    if x == n + 1:
                        return faces[1][z - 1][y - 1]
                    if y == 0:
                        return faces[2][z - 1][x - 1]
                    if y == n + 1:
                        return faces[3][z - 1][x - 1]
                    if z == 0:
                        return faces[4][y - 1][x - 1]
                    if z == n + 1:
                        return faces[5][y - 1][x - 1]
                    return blk[z - 1 - lz, y - 1 - ly, x - 1 - lx]
                rr = range(m)
                w0 = np.array([[[val(a + 1 + p, b + 1 + q, c + 1 + r) for r in rr] for q in rr]
                               for p in rr])
                wf = np.stack([
                    np.array([[val(a + 1 + p, b + 1 + q, c) for q in rr] for p in rr]),
                    np.array([[val(a + 1 + p, b + 1 + q, c + 2 * R) for q in rr] for p in rr]),
                    np.array([[val(a + 1 + p, b, c + 1 + r) for r in rr] for p in rr]),
                    np.array([[val(a + 1 + p, b + 2 * R, c + 1 + r) for r in rr] for p in rr]),
                    np.array([[val(a, b + 1 + q, c + 1 + r) for r in rr] for q in rr]),
                    np.array([[val(a + 2 * R, b + 1 + q, c + 1 + r) for r in rr] for q in rr])])
                ref = oracle.sor3d_f64(w0, wf, None, omega, 0.0, K_ITERS, 1)
                got = uu[a:a + m, b:b + m, c:c + m].cpu().numpy()
                assert np.array_equal(got[CORE, CORE, CORE].view(np.uint64),
                                      ref.u[CORE, CORE, CORE].view(np.uint64)), (K, a, b, c)
            del uu
        del u
    finally:
        ctx.close()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("ordering,name,reach", [(1, "jacobi", 1), (2, "four-colour", 3)])
def test_2d_orderings_largest_side_sampled_windows(sor, ordering, name, reach):
    """The blocked Jacobi and four-colour passes at n = 65536.  An iteration
    moves information by one cell (Jacobi) or at most three (one per colour
    sweep of the four-colour ordering), so the window oracle is exact more
    than reach * k cells inside the frozen ring; windows start at even rows
    and columns, which keeps every cell's four-colour class."""
    n = 65536
    rw = 12                          # window: interior 2 rw - 1 cells per axis
    m = 2 * rw - 1
    core = slice(reach * K_ITERS + 1, m - (reach * K_ITERS + 1))
    ctx = sor.Context(0)
    try:
        rng = np.random.default_rng(65537 + ordering)
        bdy = rng.uniform(0.0, 100.0, size=4 * n)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(19 + ordering)
        _say(f"2-D {name} n=65536: filling u0 on the device")
        u = torch.rand((n, n), dtype=torch.float64, device="cuda", generator=gen) * 100.0
        corners = [(0, 0), (0, n + 1 - 2 * rw - 1), (n + 1 - 2 * rw - 1, 0),
                   (n + 1 - 2 * rw - 1, n + 1 - 2 * rw - 1), (n // 2, n // 2 + 2),
                   (1000, 0), (0, 31000), (40002, 2)]
        top = (n + 1 - 2 * rw) & ~1        # last even corner whose ring fits
        corners = [(min(a + (a & 1), top), min(b + (b & 1), top)) for a, b in corners]
        before = {}
        for a, b in corners:
            lo_i, lo_j = max(a - 1, 0), max(b - 1, 0)
            before[(a, b)] = u[lo_i:a + 2 * rw, lo_j:b + 2 * rw].cpu().numpy().copy()
        omega = 1.0 if ordering == 1 else 2.0 / (1.0 + np.sin(np.pi / (n + 1)))
        _say(f"2-D {name} n=65536: solving")
        res = sor.solve_variant_f64(ordering, u, torch.tensor(bdy, dtype=torch.float64,
                                                              device="cuda"),
                                    None, omega, 0.0, K_ITERS, 1, hist=False, ctx=ctx)
        assert res.status == sor.NOT_CONVERGED and res.iterations == K_ITERS
        for a, b in corners:
            _say(f"2-D {name} window at ({a}, {b})")
            blk = before[(a, b)]
            lo_i, lo_j = max(a - 1, 0), max(b - 1, 0)
            val = full_value_2d(lambda i, j: blk[i - 1 - lo_i, j - 1 - lo_j], bdy, n)
            w0 = np.array([[val(a + 1 + r, b + 1 + c) for c in range(m)] for r in range(m)])
            wb = np.concatenate([[val(a, b + 1 + c) for c in range(m)],
                                 [val(a + 2 * rw, b + 1 + c) for c in range(m)],
                                 [val(a + 1 + r, b) for r in range(m)],
                                 [val(a + 1 + r, b + 2 * rw) for r in range(m)]])
            ref = oracle.variant_f64(ordering, w0, wb, None, omega, 0.0, K_ITERS, 1)
            got = u[a:a + m, b:b + m].cpu().numpy()
            assert np.array_equal(got[core, core].view(np.uint64),
                                  ref.u[core, core].view(np.uint64)), (name, a, b)
        del u
    finally:
        ctx.close()
        torch.cuda.empty_cache()
