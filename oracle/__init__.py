"""CPU oracle for red-black SOR on the 2-D 5-point heat-conduction problem.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares nothing with the GPU library: the arithmetic lives in the plain C file
``sor_oracle.c`` next to this module (FP64, no contraction, no fast-math), and
this module only marshals numpy arrays to it.

Functions follow Mittal (2014): Sec. 2.1 Eq. 1 (the SOR update), Sec. 3.1 and
Fig. 1-2 (red-black colouring, red phase first), Algorithm 1 (iteration,
check every K iterations, strict ``max change < eps`` stopping rule); the 3-D
7-point form is the extension named in Sec. 5.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sor_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsor_oracle.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, ENONFINITE = 0, 1, -1, -2, -4

_lib = None


def build(force: bool = True) -> str:
    """Compile sor_oracle.c with gcc into libsor_oracle.so (in place)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-std=c11", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_sor_f64.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int, i64p, dp, dp]
    lib.oracle_sor_f64.restype = ctypes.c_int
    lib.oracle_sor_f32.argtypes = [ctypes.c_int, fp, fp, fp, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int64,
                                   ctypes.c_int64, i64p, dp, dp]
    lib.oracle_sor_f32.restype = ctypes.c_int
    lib.oracle_residual_f64.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
    lib.oracle_residual_f64.restype = ctypes.c_int
    lib.oracle_mixed.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                 ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p, dp,
                                 dp, dp]
    lib.oracle_mixed.restype = ctypes.c_int
    lib.oracle_sor3d_f64.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int, i64p, dp, dp]
    lib.oracle_sor3d_f64.restype = ctypes.c_int
    lib.oracle_variant_f64.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                       ctypes.c_int64, i64p, dp, dp]
    lib.oracle_variant_f64.restype = ctypes.c_int
    lib.oracle_blockpar_f64.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int64, ctypes.c_int64, i64p, dp, dp]
    lib.oracle_blockpar_f64.restype = ctypes.c_int
    lib.oracle_round_half.argtypes = [ctypes.c_float]
    lib.oracle_round_half.restype = ctypes.c_float
    _lib = lib
    return lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _grid_args(n, u0, bdy, f, dtype):
    u = np.ascontiguousarray(np.array(u0, dtype=dtype).reshape(n, n))
    b = np.ascontiguousarray(np.asarray(bdy, dtype=dtype).reshape(4 * n))
    ff = None if f is None else np.ascontiguousarray(
        np.asarray(f, dtype=dtype).reshape(n, n))
    return u, b, ff


@dataclass
class SorResult:
    u: np.ndarray            # final n x n interior
    status: int              # OK / NOT_CONVERGED / ENONFINITE
    iterations: int          # iteration whose check passed, else max_iters
    final_max_delta: float   # max change of the last checked iteration
    mhist: np.ndarray | None  # max change of every iteration run

    @property
    def converged(self) -> bool:
        return self.status == OK


def sor_f64(u0, bdy, f, omega, tol, max_iters, check_every=1, threads=1,
            hist=False) -> SorResult:
    """FP64 red-black SOR (Eq. 1 with red-black ordering, Algorithm 1)."""
    lib = _load()
    n = int(np.asarray(bdy).size // 4)
    u, b, ff = _grid_args(n, u0, bdy, f, np.float64)
    it = ctypes.c_int64(0)
    mx = ctypes.c_double(0.0)
    mh = np.zeros(max_iters, dtype=np.float64) if hist else None
    st = lib.oracle_sor_f64(n, _ptr(u, ctypes.c_double), _ptr(b, ctypes.c_double),
                            _ptr(ff, ctypes.c_double), float(omega), float(tol),
                            int(max_iters), int(check_every), int(threads),
                            ctypes.byref(it), ctypes.byref(mx),
                            _ptr(mh, ctypes.c_double))
    if st < 0 and st != ENONFINITE:
        raise ValueError(f"oracle_sor_f64 rejected its arguments (status {st})")
    if mh is not None:
        mh = mh[: it.value]
    return SorResult(u, st, it.value, mx.value, mh)


def sor_f32(u0, bdy, f, omega, tol, max_iters, check_every=1,
            hist=False) -> SorResult:
    """Red-black SOR with float storage and float arithmetic."""
    lib = _load()
    n = int(np.asarray(bdy).size // 4)
    u, b, ff = _grid_args(n, u0, bdy, f, np.float32)
    it = ctypes.c_int64(0)
    mx = ctypes.c_double(0.0)
    mh = np.zeros(max_iters, dtype=np.float64) if hist else None
    st = lib.oracle_sor_f32(n, _ptr(u, ctypes.c_float), _ptr(b, ctypes.c_float),
                            _ptr(ff, ctypes.c_float), float(omega), float(tol),
                            int(max_iters), int(check_every), ctypes.byref(it),
                            ctypes.byref(mx), _ptr(mh, ctypes.c_double))
    if st < 0 and st != ENONFINITE:
        raise ValueError(f"oracle_sor_f32 rejected its arguments (status {st})")
    if mh is not None:
        mh = mh[: it.value]
    return SorResult(u, st, it.value, mx.value, mh)


def residual_f64(u, bdy, f=None):
    """Return (r, sum r^2, sum b^2, max|r|) of the h*h-scaled 5-point system."""
    lib = _load()
    n = int(np.asarray(bdy).size // 4)
    uu, b, ff = _grid_args(n, u, bdy, f, np.float64)
    r = np.zeros((n, n), dtype=np.float64)
    stats = np.zeros(3, dtype=np.float64)
    st = lib.oracle_residual_f64(n, _ptr(uu, ctypes.c_double),
                                 _ptr(b, ctypes.c_double),
                                 _ptr(ff, ctypes.c_double),
                                 _ptr(r, ctypes.c_double),
                                 _ptr(stats, ctypes.c_double))
    if st != OK:
        raise ValueError(f"oracle_residual_f64 failed (status {st})")
    return r, float(stats[0]), float(stats[1]), float(stats[2])


def rel_residual(u, bdy, f=None) -> float:
    _, sr, sb, _ = residual_f64(u, bdy, f)
    return float(np.sqrt(sr) / np.sqrt(sb)) if sb > 0 else float(np.sqrt(sr))


@dataclass
class MixedResult:
    u: np.ndarray
    status: int
    outer_steps: int
    rel_residual: float
    relhist: np.ndarray
    last_correction: float = float("nan")

    @property
    def converged(self) -> bool:
        return self.status == OK


def mixed(u0, bdy, f, omega, rel_tol, max_outer, inner_bits=32,
          inner_iters=None, corr_tol=0.0, threads=1) -> MixedResult:
    """FP64 defect correction around reduced-precision red-black SOR
    (threads > 1: inner half-sweeps on that many OpenMP workers, same result)."""
    lib = _load()
    n = int(np.asarray(bdy).size // 4)
    if inner_iters is None:
        inner_iters = (max(1, n // 2) + 5) // 6 * 6     # the library's default count
    u, b, ff = _grid_args(n, u0, bdy, f, np.float64)
    outer = ctypes.c_int64(0)
    rel = ctypes.c_double(0.0)
    rh = np.zeros(max_outer + 1, dtype=np.float64)
    corr = ctypes.c_double(0.0)
    st = lib.oracle_mixed(n, _ptr(u, ctypes.c_double), _ptr(b, ctypes.c_double),
                          _ptr(ff, ctypes.c_double), float(omega), float(rel_tol),
                          float(corr_tol), int(max_outer), int(inner_bits),
                          int(inner_iters), int(threads), ctypes.byref(outer),
                          ctypes.byref(rel),
                          _ptr(rh, ctypes.c_double), ctypes.byref(corr))
    if st < 0 and st != ENONFINITE:
        raise ValueError(f"oracle_mixed rejected its arguments (status {st})")
    return MixedResult(u, st, outer.value, rel.value, rh[: outer.value + 1],
                       corr.value)


ORDER_JACOBI = 1
ORDER_FOUR_COLOUR = 2


def variant_f64(ordering, u0, bdy, f, omega, tol, max_iters, check_every=1,
                hist=False) -> SorResult:
    """FP64 Jacobi (ordering 1: every cell from the previous iterate, w = 1
    plain Jacobi) or four-colour SOR (ordering 2: colours 2*(i mod 2) + (j mod
    2) of the full array updated in the order 0, 1, 2, 3), same update, stop
    rule and array conventions as sor_f64."""
    lib = _load()
    n = int(np.asarray(bdy).size // 4)
    u, b, ff = _grid_args(n, u0, bdy, f, np.float64)
    it = ctypes.c_int64(0)
    mx = ctypes.c_double(0.0)
    mh = np.zeros(max_iters, dtype=np.float64) if hist else None
    st = lib.oracle_variant_f64(int(ordering), n, _ptr(u, ctypes.c_double),
                                _ptr(b, ctypes.c_double), _ptr(ff, ctypes.c_double),
                                float(omega), float(tol), int(max_iters), int(check_every),
                                ctypes.byref(it), ctypes.byref(mx), _ptr(mh, ctypes.c_double))
    if st < 0 and st != ENONFINITE:
        raise ValueError(f"oracle_variant_f64 rejected its arguments (status {st})")
    if mh is not None:
        mh = mh[: it.value]
    return SorResult(u, st, it.value, mx.value, mh)


def blockpar_f64(u0, bdy, f, omega, block_rows, block_cols, tol, max_iters,
                 check_every=1, hist=False) -> SorResult:
    """FP64 block-parallel SOR (the form Sec. 3.1 names): blocks of block_rows
    x block_cols interior cells, aligned at cell (1, 1), each updated by one
    red-black SOR iteration per iteration with every neighbour outside the
    block taken at the previous iterate.  Stop rule and array conventions as
    sor_f64."""
    lib = _load()
    n = int(np.asarray(bdy).size // 4)
    u, b, ff = _grid_args(n, u0, bdy, f, np.float64)
    it = ctypes.c_int64(0)
    mx = ctypes.c_double(0.0)
    mh = np.zeros(max_iters, dtype=np.float64) if hist else None
    st = lib.oracle_blockpar_f64(n, _ptr(u, ctypes.c_double), _ptr(b, ctypes.c_double),
                                 _ptr(ff, ctypes.c_double), float(omega), int(block_rows),
                                 int(block_cols), float(tol), int(max_iters),
                                 int(check_every), ctypes.byref(it), ctypes.byref(mx),
                                 _ptr(mh, ctypes.c_double))
    if st < 0 and st != ENONFINITE:
        raise ValueError(f"oracle_blockpar_f64 rejected its arguments (status {st})")
    if mh is not None:
        mh = mh[: it.value]
    return SorResult(u, st, it.value, mx.value, mh)


def sor3d_f64(u0, bdy, f, omega, tol, max_iters, check_every=1, threads=1,
              hist=False) -> SorResult:
    """FP64 red-black SOR on the 7-point stencil of the unit cube: u0 is
    (n, n, n) indexed [z][y][x], bdy (6, n, n) holds the faces x = 0, x = n+1
    ([z][y]), y = 0, y = n+1 ([z][x]), z = 0, z = n+1 ([y][x])."""
    lib = _load()
    b = np.ascontiguousarray(np.asarray(bdy, dtype=np.float64).reshape(-1))
    n = int(round((b.size // 6) ** 0.5))
    if 6 * n * n != b.size:
        raise ValueError("bdy must hold 6 faces of n*n values")
    u = np.ascontiguousarray(np.array(u0, dtype=np.float64).reshape(n, n, n))
    ff = None if f is None else np.ascontiguousarray(
        np.asarray(f, dtype=np.float64).reshape(n, n, n))
    it = ctypes.c_int64(0)
    mx = ctypes.c_double(0.0)
    mh = np.zeros(max_iters, dtype=np.float64) if hist else None
    st = lib.oracle_sor3d_f64(n, _ptr(u, ctypes.c_double), _ptr(b, ctypes.c_double),
                              _ptr(ff, ctypes.c_double), float(omega), float(tol),
                              int(max_iters), int(check_every), int(threads),
                              ctypes.byref(it), ctypes.byref(mx),
                              _ptr(mh, ctypes.c_double))
    if st < 0 and st != ENONFINITE:
        raise ValueError(f"oracle_sor3d_f64 rejected its arguments (status {st})")
    if mh is not None:
        mh = mh[: it.value]
    return SorResult(u, st, it.value, mx.value, mh)


def round_half(x: float) -> float:
    """IEEE binary16 rounding (ties to even) of a float, returned as float."""
    return float(_load().oracle_round_half(float(x)))
