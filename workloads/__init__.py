"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws numbers and fixes problem parameters; it contains none
of the solver's arithmetic.  Both the CPU oracle and the GPU library receive
exactly these arrays.

Random streams: ``numpy.random.default_rng(seed)`` (PCG64).  Draw order for a
grid: boundary edges north, south, west, east (one draw of 4n values), then
the source f row-major.  For batches and request streams the per-item draws are
taken in item order: side length, then boundary, then f.

Workloads (sizes are interior nodes per side; h = 1/(n+1)):
  * ``laplace_top_edge`` -- Laplace, north edge = value, other edges 0,
    interior 0 (the paper's heat-conduction set-up, Sec. 3.4).
  * ``laplace_random_boundary`` -- Laplace, each boundary node U[0, 100].
  * ``poisson_manufactured`` -- -lap u = f with f i.i.d. N(0,1) plus the
    manufactured term 2 pi^2 sin(pi x) sin(pi y), zero boundary.
  * ``batch_grids`` -- many grids with log-uniform side lengths.
  * ``ServingStream`` -- seeded Poisson arrivals of solve requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def omega_opt(n: int) -> float:
    """Young's optimal relaxation factor 2 / (1 + sin(pi h)), h = 1/(n+1)."""
    return 2.0 / (1.0 + math.sin(math.pi / (n + 1)))


@dataclass
class Grid:
    n: int
    u0: np.ndarray              # n x n initial interior (float64)
    bdy: np.ndarray             # 4n boundary values: N, S, W, E (float64)
    f: np.ndarray | None        # n x n source, or None for Laplace
    omega: float
    tol: float = 1e-8
    max_iters: int = 100000
    check_every: int = 1
    meta: dict = field(default_factory=dict)


def laplace_top_edge(n: int = 256, top: float = 100.0, tol: float = 1e-6,
                     max_iters: int = 5000, check_every: int = 1) -> Grid:
    bdy = np.zeros(4 * n, dtype=np.float64)
    bdy[:n] = top
    return Grid(n, np.zeros((n, n)), bdy, None, omega_opt(n), tol, max_iters,
                check_every, {"name": f"laplace_top_edge_{n}"})


def laplace_random_boundary(n: int = 4096, seed: int = 2, tol: float = 1e-8,
                            max_iters: int = 1000, check_every: int = 10) -> Grid:
    rng = np.random.default_rng(seed)
    bdy = rng.uniform(0.0, 100.0, size=4 * n)
    return Grid(n, np.zeros((n, n)), bdy, None, omega_opt(n), tol, max_iters,
                check_every, {"name": f"laplace_random_boundary_{n}", "seed": seed})


def manufactured_term(n: int) -> np.ndarray:
    """2 pi^2 sin(pi x_j) sin(pi y_i) on the interior nodes x_j = j h, y_i = i h."""
    h = 1.0 / (n + 1)
    s = np.sin(np.pi * h * np.arange(1, n + 1))
    return 2.0 * np.pi ** 2 * np.outer(s, s)


def poisson_manufactured(n: int = 4096, seed: int = 3, noise: bool = True) -> Grid:
    rng = np.random.default_rng(seed)
    bdy = np.zeros(4 * n, dtype=np.float64)
    f = manufactured_term(n)
    if noise:
        f = f + rng.standard_normal((n, n))
    return Grid(n, np.zeros((n, n)), bdy, f, omega_opt(n), 1e-10, 100000, 1,
                {"name": f"poisson_manufactured_{n}", "seed": seed})


def random_grid(rng: np.random.Generator, n: int, with_f: bool,
                tol: float = 1e-8) -> Grid:
    bdy = rng.uniform(0.0, 100.0, size=4 * n)
    f = rng.standard_normal((n, n)) if with_f else None
    return Grid(n, np.zeros((n, n)), bdy, f, omega_opt(n), tol, 1000000, 1)


def batch_grids(count: int = 512, lo: int = 64, hi: int = 1024, seed: int = 4,
                tol: float = 1e-8) -> list[Grid]:
    """count grids, side n = round(exp(U(ln lo, ln hi))), f on odd indices."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(count):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        grid = random_grid(rng, n, with_f=(g % 2 == 1), tol=tol)
        grid.meta = {"index": g}
        out.append(grid)
    return out


def random_small(seed: int, n: int, with_f: bool = True, omega: float | None = None,
                 nonzero_u0: bool = False) -> Grid:
    """Small seeded grid for parity tests (random boundary, f, optional u0)."""
    rng = np.random.default_rng(seed)
    bdy = rng.uniform(0.0, 100.0, size=4 * n)
    f = rng.standard_normal((n, n)) * 1000.0 if with_f else None
    u0 = rng.uniform(0.0, 100.0, size=(n, n)) if nonzero_u0 else np.zeros((n, n))
    return Grid(n, u0, bdy, f, omega_opt(n) if omega is None else omega)


def random_cube(seed: int, n: int, with_f: bool = True, omega: float | None = None,
                nonzero_u0: bool = False, bdy_scale: float = 100.0) -> Grid:
    """Seeded 3-D grid of side n: boundary (6, n, n) U[0, bdy_scale] (faces
    x = 0, x = n+1, y = 0, y = n+1, z = 0, z = n+1), source f (n, n, n) of
    N(0, 1000^2) values or None, u0 (n, n, n) zero or U[0, 100]."""
    rng = np.random.default_rng([seed, 3])
    bdy = rng.uniform(0.0, bdy_scale, size=(6, n, n))
    f = rng.standard_normal((n, n, n)) * 1000.0 if with_f else None
    u0 = rng.uniform(0.0, 100.0, size=(n, n, n)) if nonzero_u0 else np.zeros((n, n, n))
    return Grid(n, u0, bdy, f, omega_opt(n) if omega is None else omega, meta={"dims": 3})


class ServingStream:
    """Seeded Poisson arrivals of solve requests, generated on demand.

    Request k has side n = round(exp(U(ln lo, ln hi))), boundary values
    U[0, 100] (4n, order north, south, west, east) and a source f that is an
    n x n window, at a seeded offset, of one of a few pre-drawn hi x hi fields
    of i.i.d. N(0, 1) values (so every f is itself i.i.d. N(0, 1) and no
    request costs a fresh hi^2 draw).  Arrival gaps are exponential with mean
    1/rate."""

    def __init__(self, count=2000, rate_per_s=100.0, lo=128, hi=2048, seed=5,
                 pool=4):
        self.count, self.rate, self.lo, self.hi, self.seed = count, rate_per_s, lo, hi, seed
        rng = np.random.default_rng([seed, 0])
        self.pool = [rng.standard_normal((hi, hi)) for _ in range(pool)]
        arr = np.random.default_rng([seed, 1])
        gaps = arr.exponential(1.0 / rate_per_s, size=count)
        self.arrivals = np.cumsum(gaps)
        sz = np.random.default_rng([seed, 2])
        self.sizes = [int(round(math.exp(x))) for x in
                      sz.uniform(math.log(lo), math.log(hi), size=count)]

    def request(self, k):
        """(n, boundary, f) of request k."""
        n = self.sizes[k]
        rng = np.random.default_rng([self.seed, 3, k])
        bdy = rng.uniform(0.0, 100.0, size=4 * n)
        field = self.pool[k % len(self.pool)]
        oi, oj = (int(x) for x in rng.integers(0, self.hi - n + 1, size=2))
        f = np.ascontiguousarray(field[oi:oi + n, oj:oj + n])
        return n, bdy, f
