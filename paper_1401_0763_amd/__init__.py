"""Red-black SOR for AMD MI355X (gfx950): Python binding of libsor.

Thin ctypes marshalling over the C ABI in ``include/sor.h``; every step of a
solve runs in the library's HIP kernels.  PyTorch supplies device memory and
streams only: arrays are torch tensors on a ROCm device, passed by data
pointer, and work is ordered on ``torch.cuda.current_stream()``.

The library must have been built (``python -m paper_1401_0763_amd.build`` or
``__graft_entry__.build()``); importing the solver functions without it raises.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsor.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EBUSY, ETIMEOUT = (
    0, 1, -1, -2, -3, -4, -5, -6)
KERNEL_BLOCKED, KERNEL_SIMPLE = 0, 1

_STATUS_NAMES = {OK: "OK", NOT_CONVERGED: "NOT_CONVERGED", EINVAL: "EINVAL",
                 ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENONFINITE: "ENONFINITE",
                 EBUSY: "EBUSY", ETIMEOUT: "ETIMEOUT"}


class SorError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64),
                ("final_max_delta", ctypes.c_double),
                ("converged", ctypes.c_int32),
                ("outer_steps", ctypes.c_int32),
                ("rel_residual", ctypes.c_double),
                ("passes", ctypes.c_int64),
                ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _MixedDesc(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("boundary", ctypes.c_void_p),
                ("rhs", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("omega", ctypes.c_double),
                ("rel_tol", ctypes.c_double), ("corr_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int64), ("inner_iters", ctypes.c_int64)]


class _Request(ctypes.Structure):
    _fields_ = [("u0", ctypes.c_void_p), ("boundary", ctypes.c_void_p),
                ("rhs", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("omega", ctypes.c_double),
                ("rel_tol", ctypes.c_double), ("corr_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int64), ("inner_iters", ctypes.c_int64)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("result", _Result), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class _GridDesc(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("boundary", ctypes.c_void_p),
                ("rhs", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("omega", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iters", ctypes.c_int64),
                ("check_every", ctypes.c_int64)]


class _Tiling(ctypes.Structure):
    _fields_ = [("iters_per_pass", ctypes.c_int32), ("seg_rows", ctypes.c_int32)]


@dataclass
class Result:
    status: int
    iterations: int
    final_max_delta: float
    converged: bool
    outer_steps: int
    rel_residual: float
    passes: int
    hist: list | None = None


_lib = None
_lock = threading.Lock()


def _declare(lib):
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.sor_version.restype = ctypes.c_char_p
    lib.sor_version.argtypes = []
    lib.sor_omega_opt.restype = ctypes.c_double
    lib.sor_omega_opt.argtypes = [ctypes.c_int32]
    lib.sor_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    lib.sor_ctx_create.restype = ctypes.c_int
    lib.sor_ctx_destroy.argtypes = [P]
    lib.sor_ctx_destroy.restype = None
    lib.sor_last_error.argtypes = [P]
    lib.sor_last_error.restype = ctypes.c_char_p
    lib.sor_ctx_set_profiling.argtypes = [P, i32]
    lib.sor_ctx_set_profiling.restype = ctypes.c_int
    lib.sor_ctx_get_profile.argtypes = [P, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.sor_ctx_get_profile.restype = ctypes.c_int
    lib.sor_ctx_set_kernel.argtypes = [P, i32]
    lib.sor_ctx_set_kernel.restype = ctypes.c_int
    lib.sor_ctx_set_tiling.argtypes = [P, i32, ctypes.POINTER(_Tiling)]
    lib.sor_ctx_set_tiling.restype = ctypes.c_int
    lib.sor_ctx_get_tiling.argtypes = [P, i32, ctypes.POINTER(_Tiling)]
    lib.sor_ctx_get_tiling.restype = ctypes.c_int
    lib.sor_ctx_tiling_for.argtypes = [P, i32, i32, i32, ctypes.POINTER(_Tiling)]
    lib.sor_ctx_tiling_for.restype = ctypes.c_int
    solve_args = [P, P, P, P, i32, dbl, dbl, i64, i64, P,
                  ctypes.POINTER(_Result), P]
    for name in ("sor_solve_f64", "sor_solve_f32", "sor_solve3d_f64",
                 "sor_solve_f64_noalloc"):
        getattr(lib, name).argtypes = solve_args
        getattr(lib, name).restype = ctypes.c_int
    lib.sor_batch_last_times.argtypes = [P, i32, P]
    lib.sor_batch_last_times.restype = ctypes.c_int
    lib.sor_solve_variant_f64.argtypes = [P, i32] + solve_args[1:]
    lib.sor_solve_variant_f64.restype = ctypes.c_int
    lib.sor_solve_blockpar_f64.argtypes = [P, P, P, P, i32, dbl, i32, i32, dbl, i64, i64, P,
                                           ctypes.POINTER(_Result), P]
    lib.sor_solve_blockpar_f64.restype = ctypes.c_int
    lib.sor_ctx_set_variant_tiling.argtypes = [P, i32, ctypes.POINTER(_Tiling)]
    lib.sor_ctx_set_variant_tiling.restype = ctypes.c_int
    lib.sor_ctx_get_variant_tiling.argtypes = [P, i32, ctypes.POINTER(_Tiling)]
    lib.sor_ctx_get_variant_tiling.restype = ctypes.c_int
    lib.sor_ctx_set_tiling3d.argtypes = [P, i32, i32, i32, i32]
    lib.sor_ctx_set_tiling3d.restype = ctypes.c_int
    pi32 = ctypes.POINTER(ctypes.c_int32)
    lib.sor_ctx_tiling3d_for.argtypes = [P, i32, i32, i64, pi32, pi32, pi32, pi32]
    lib.sor_ctx_tiling3d_for.restype = ctypes.c_int
    lib.sor_residual_f64.argtypes = [P, P, P, P, i32, P, P, P]
    lib.sor_residual_f64.restype = ctypes.c_int
    lib.sor_solve_mixed.argtypes = [P, P, P, P, i32, dbl, dbl, i64, i32, i64, P,
                                    ctypes.POINTER(_Result), P]
    lib.sor_solve_mixed.restype = ctypes.c_int
    lib.sor_batch_solve_f64.argtypes = [P, ctypes.POINTER(_GridDesc), i32, P,
                                        ctypes.POINTER(_Result)]
    lib.sor_batch_solve_f64.restype = ctypes.c_int
    lib.sor_autotune.argtypes = [P, i32, i32, ctypes.POINTER(_Tiling)]
    lib.sor_autotune.restype = ctypes.c_int
    lib.sor_autotune_batch.argtypes = [P, i32, i32, ctypes.POINTER(_Tiling)]
    lib.sor_autotune_batch.restype = ctypes.c_int
    lib.sor_batch_solve_mixed.argtypes = [P, ctypes.POINTER(_MixedDesc), i32, i32, P,
                                          ctypes.POINTER(_Result)]
    lib.sor_batch_solve_mixed.restype = ctypes.c_int
    lib.sor_server_create.argtypes = [ctypes.c_int, i32, ctypes.c_size_t, i32, dbl,
                                      ctypes.POINTER(P)]
    lib.sor_server_create.restype = ctypes.c_int
    lib.sor_server_submit.argtypes = [P, ctypes.POINTER(_Request),
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.sor_server_submit.restype = ctypes.c_int
    lib.sor_server_poll.argtypes = [P, ctypes.c_uint64, dbl, ctypes.POINTER(_RequestInfo), P]
    lib.sor_server_poll.restype = ctypes.c_int
    lib.sor_server_clock.argtypes = [P]
    lib.sor_server_clock.restype = dbl
    lib.sor_server_stats.argtypes = [P] + [ctypes.POINTER(i64)] * 4
    lib.sor_server_stats.restype = ctypes.c_int
    lib.sor_server_memory.argtypes = [P] + [ctypes.POINTER(ctypes.c_size_t)] * 3
    lib.sor_server_memory.restype = ctypes.c_int
    lib.sor_server_last_error.argtypes = [P]
    lib.sor_server_last_error.restype = ctypes.c_char_p
    lib.sor_server_destroy.argtypes = [P]
    lib.sor_server_destroy.restype = None


def load_library():
    """Load libsor.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_1401_0763_amd.build`")
            lib = ctypes.CDLL(LIB_PATH)
            _declare(lib)
            _lib = lib
    return _lib


def version() -> str:
    return load_library().sor_version().decode()


def omega_opt(n: int) -> float:
    """Young's optimal relaxation factor for side n (sor_omega_opt)."""
    return load_library().sor_omega_opt(int(n))


class Context:
    """A libsor context bound to one device (owns the working grids)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.sor_ctx_create(int(device), ctypes.byref(h))
        if st != OK:
            raise SorError(st, f"sor_ctx_create(device={device}) failed")
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sor_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return self.lib.sor_last_error(self.handle).decode()

    def _check(self, st, allow=(OK, NOT_CONVERGED)):
        if st not in allow:
            raise SorError(st, self.error())
        return st

    def set_tiling3d(self, cx: int = 0, cy: int = 0, zs: int = 0, iters: int = 0):
        """3-D streaming kernel: core tile sizes and iterations per launch
        (0: automatic)."""
        self._check(self.lib.sor_ctx_set_tiling3d(self.handle, int(iters), int(cx), int(cy),
                                                  int(zs)))

    def tiling3d_for(self, n: int, has_rhs: bool = False, check_every: int = 1):
        """(iters_per_launch, cx, cy, zs) a 3-D solve of side n would use."""
        t, a, b, z = (ctypes.c_int32() for _ in range(4))
        self._check(self.lib.sor_ctx_tiling3d_for(self.handle, int(n), int(bool(has_rhs)),
                                                  int(check_every), ctypes.byref(t),
                                                  ctypes.byref(a), ctypes.byref(b),
                                                  ctypes.byref(z)))
        return t.value, a.value, b.value, z.value

    def set_kernel(self, kernel: int):
        self._check(self.lib.sor_ctx_set_kernel(self.handle, int(kernel)))

    def set_profiling(self, on: bool):
        self._check(self.lib.sor_ctx_set_profiling(self.handle, int(bool(on))))

    def profile(self) -> tuple[float, int]:
        """(total sweep-kernel milliseconds, timed launches) since profiling
        was switched on; each run of launches between host checks is timed as
        a whole."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        self._check(self.lib.sor_ctx_get_profile(self.handle, ctypes.byref(ms),
                                                 ctypes.byref(k)))
        return ms.value, k.value

    def set_tiling(self, bits: int, iters_per_pass: int = 0, seg_rows: int = 0):
        t = _Tiling(int(iters_per_pass), int(seg_rows))
        self._check(self.lib.sor_ctx_set_tiling(self.handle, int(bits), ctypes.byref(t)))

    def autotune(self, bits: int, n: int) -> tuple[int, int]:
        """Time candidate tilings for an n x n grid; returns (iters_per_pass,
        seg_rows) and records it for n's size class."""
        t = _Tiling()
        self._check(self.lib.sor_autotune(self.handle, int(bits), int(n), ctypes.byref(t)))
        return t.iters_per_pass, t.seg_rows

    def batch_times(self, count: int) -> list[float]:
        """Retire time (ms after the persistent launch began) of each grid of
        the most recent batch_solve_f64 on this context."""
        out = (ctypes.c_double * int(count))()
        self._check(self.lib.sor_batch_last_times(self.handle, int(count), out), (OK,))
        return list(out)

    def autotune_batch(self, bits: int, n: int) -> tuple[int, int]:
        """Time candidate tilings on a scratch batch of n x n grids; returns
        (iters_per_pass, seg_rows) and records it for batched solves of n's
        size class."""
        t = _Tiling()
        self._check(self.lib.sor_autotune_batch(self.handle, int(bits), int(n),
                                                ctypes.byref(t)))
        return t.iters_per_pass, t.seg_rows

    def set_variant_tiling(self, ordering: int, iters_per_pass: int = 0, seg_rows: int = 0):
        """Tiling of the blocked kernel of ORDER_FOUR_COLOUR, ORDER_JACOBI or
        ORDER_BLOCK_PARALLEL (0 keeps a field)."""
        t = _Tiling(int(iters_per_pass), int(seg_rows))
        self._check(self.lib.sor_ctx_set_variant_tiling(self.handle, int(ordering),
                                                        ctypes.byref(t)))

    def get_variant_tiling(self, ordering: int) -> tuple[int, int]:
        """The blocked tiling of an ordering; seg_rows 0 means chosen per grid size."""
        t = _Tiling()
        self._check(self.lib.sor_ctx_get_variant_tiling(self.handle, int(ordering),
                                                        ctypes.byref(t)))
        return t.iters_per_pass, t.seg_rows

    def get_tiling(self, bits: int) -> tuple[int, int]:
        """The context's tiling; 0 means chosen per solve (iters_per_pass by
        the pass kernel's occupancy, seg_rows by the grid side)."""
        t = _Tiling()
        self._check(self.lib.sor_ctx_get_tiling(self.handle, int(bits), ctypes.byref(t)))
        return t.iters_per_pass, t.seg_rows

    def tiling_for(self, bits: int, n: int, has_rhs: bool = False) -> tuple[int, int]:
        """The (iters_per_pass, seg_rows) a plain solve of side n would use."""
        t = _Tiling()
        self._check(self.lib.sor_ctx_tiling_for(self.handle, int(bits), int(n),
                                                int(bool(has_rhs)), ctypes.byref(t)))
        return t.iters_per_pass, t.seg_rows


_contexts: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    """Per-device default context (created on first use)."""
    import torch
    if device is None:
        device = torch.cuda.current_device()
    with _lock:
        ctx = _contexts.get(device)
    if ctx is None:
        ctx = Context(device)
        with _lock:
            _contexts[device] = ctx
    return ctx


def _stream_handle(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_tensor(name, t, dtype, shape):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _result(st, r: _Result, hist=None) -> Result:
    return Result(st, r.iterations, r.final_max_delta, bool(r.converged),
                  r.outer_steps, r.rel_residual, r.passes, hist)


@dataclass
class GridSpec:
    """One grid of a batched solve (torch float64 CUDA tensors)."""
    u: object                 # n x n, solved in place
    boundary: object          # 4n
    rhs: object = None        # n x n or None
    omega: float | None = None
    tol: float = 1e-8
    max_iters: int = 1000000
    check_every: int = 1


def batch_solve_f64(specs, ctx: Context | None = None) -> list[Result]:
    """Solve many grids in one persistent launch; one Result per grid."""
    import torch
    specs = list(specs)
    if not specs:
        return []
    ctx = ctx or context(specs[0].u.device.index)
    descs = (_GridDesc * len(specs))()
    for k, sp in enumerate(specs):
        n = sp.u.shape[0]
        d = descs[k]
        d.u = _check_tensor("u", sp.u, torch.float64, (n, n))
        d.boundary = _check_tensor("boundary", sp.boundary, torch.float64, (4 * n,))
        d.rhs = None if sp.rhs is None else _check_tensor("rhs", sp.rhs, torch.float64, (n, n))
        d.n = n
        d.omega = omega_opt(n) if sp.omega is None else sp.omega
        d.tol = sp.tol
        d.max_iters = sp.max_iters
        d.check_every = sp.check_every
    res = (_Result * len(specs))()
    st = ctx.lib.sor_batch_solve_f64(ctx.handle, descs, len(specs),
                                     _stream_handle(specs[0].u), res)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    return [_result(r.status, r) for r in res]


def _solve_plain(fn, dtype, u, boundary, rhs, omega, tol, max_iters,
                 check_every, hist, ctx):
    n = u.shape[0]
    pu = _check_tensor("u", u, dtype, (n, n))
    pb = _check_tensor("boundary", boundary, dtype, (4 * n,))
    pf = None if rhs is None else _check_tensor("rhs", rhs, dtype, (n, n))
    ctx = ctx or context(u.device.index)
    res = _Result()
    hbuf = (ctypes.c_double * int(max_iters))() if hist else None
    st = fn(ctx.handle, pu, pb, pf, int(n), float(omega), float(tol),
            int(max_iters), int(check_every), _stream_handle(u),
            ctypes.byref(res), hbuf)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    h = list(hbuf[: res.iterations]) if hist else None
    return _result(st, res, h)


def solve_f64(u, boundary, rhs=None, omega=None, tol=1e-8, max_iters=100000,
              check_every=1, hist=False, ctx: Context | None = None) -> Result:
    """FP64 red-black SOR in place on u (n x n float64 CUDA tensor)."""
    import torch
    n = u.shape[0]
    if omega is None:
        omega = omega_opt(n)
    ctx = ctx or context(u.device.index)
    return _solve_plain(ctx.lib.sor_solve_f64, torch.float64, u, boundary, rhs,
                        omega, tol, max_iters, check_every, hist, ctx)


def solve_f64_noalloc(u, boundary, rhs=None, omega=None, tol=1e-8, max_iters=100000,
                      check_every=1, hist=False, ctx: Context | None = None) -> Result:
    """solve_f64 through sor_solve_f64_noalloc: the library allocates no
    device memory for the call (working grids in its fixed per-GPU region;
    n <= 1951 Laplace, n <= 1583 with a source)."""
    import torch
    n = u.shape[0]
    if omega is None:
        omega = omega_opt(n)
    ctx = ctx or context(u.device.index)
    return _solve_plain(ctx.lib.sor_solve_f64_noalloc, torch.float64, u, boundary, rhs,
                        omega, tol, max_iters, check_every, hist, ctx)


def solve_f32(u, boundary, rhs=None, omega=None, tol=1e-5, max_iters=100000,
              check_every=1, hist=False, ctx: Context | None = None) -> Result:
    """Float-storage red-black SOR in place on u (n x n float32 CUDA tensor)."""
    import torch
    n = u.shape[0]
    if omega is None:
        omega = omega_opt(n)
    ctx = ctx or context(u.device.index)
    return _solve_plain(ctx.lib.sor_solve_f32, torch.float32, u, boundary, rhs,
                        omega, tol, max_iters, check_every, hist, ctx)


ORDER_RED_BLACK, ORDER_JACOBI, ORDER_FOUR_COLOUR, ORDER_BLOCK_PARALLEL = 0, 1, 2, 3


def solve_variant_f64(ordering, u, boundary, rhs=None, omega=None, tol=1e-8,
                      max_iters=100000, check_every=1, hist=False,
                      ctx: Context | None = None) -> Result:
    """FP64 solve in place on u with the given ordering (ORDER_RED_BLACK,
    ORDER_JACOBI or ORDER_FOUR_COLOUR); otherwise as solve_f64."""
    import torch
    n = u.shape[0]
    if omega is None:
        omega = 1.0 if ordering == ORDER_JACOBI else omega_opt(n)
    pu = _check_tensor("u", u, torch.float64, (n, n))
    pb = _check_tensor("boundary", boundary, torch.float64, (4 * n,))
    pf = None if rhs is None else _check_tensor("rhs", rhs, torch.float64, (n, n))
    ctx = ctx or context(u.device.index)
    res = _Result()
    hbuf = (ctypes.c_double * int(max_iters))() if hist else None
    st = ctx.lib.sor_solve_variant_f64(ctx.handle, int(ordering), pu, pb, pf, int(n),
                                       float(omega), float(tol), int(max_iters),
                                       int(check_every), _stream_handle(u),
                                       ctypes.byref(res), hbuf)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    h = list(hbuf[: res.iterations]) if hist else None
    return _result(st, res, h)


def solve_blockpar_f64(u, boundary, block_rows, block_cols, rhs=None, omega=1.0, tol=1e-8,
                       max_iters=100000, check_every=1, hist=False,
                       ctx: Context | None = None) -> Result:
    """FP64 block-parallel SOR in place on u: blocks of block_rows x
    block_cols interior cells, each updated per iteration by one red-black
    iteration with neighbours in other blocks at the previous iterate;
    otherwise as solve_f64.  The default omega is 1 (the method does not
    converge for every omega in (0, 2))."""
    import torch
    n = u.shape[0]
    pu = _check_tensor("u", u, torch.float64, (n, n))
    pb = _check_tensor("boundary", boundary, torch.float64, (4 * n,))
    pf = None if rhs is None else _check_tensor("rhs", rhs, torch.float64, (n, n))
    ctx = ctx or context(u.device.index)
    res = _Result()
    hbuf = (ctypes.c_double * int(max_iters))() if hist else None
    st = ctx.lib.sor_solve_blockpar_f64(ctx.handle, pu, pb, pf, int(n), float(omega),
                                        int(block_rows), int(block_cols), float(tol),
                                        int(max_iters), int(check_every), _stream_handle(u),
                                        ctypes.byref(res), hbuf)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    h = list(hbuf[: res.iterations]) if hist else None
    return _result(st, res, h)


def solve3d_f64(u, boundary, rhs=None, omega=None, tol=1e-8, max_iters=100000,
                check_every=1, hist=False, ctx: Context | None = None) -> Result:
    """FP64 red-black SOR on the 7-point stencil of the unit cube, in place on
    u (n x n x n float64 CUDA tensor indexed [z][y][x]); boundary (6, n, n)
    holds the faces x = 0, x = n+1 ([z][y]), y = 0, y = n+1 ([z][x]),
    z = 0, z = n+1 ([y][x]); rhs (n, n, n) or None."""
    import torch
    n = u.shape[0]
    if omega is None:
        omega = omega_opt(n)
    pu = _check_tensor("u", u, torch.float64, (n, n, n))
    pb = _check_tensor("boundary", boundary, torch.float64, (6, n, n))
    pf = None if rhs is None else _check_tensor("rhs", rhs, torch.float64, (n, n, n))
    ctx = ctx or context(u.device.index)
    res = _Result()
    hbuf = (ctypes.c_double * int(max_iters))() if hist else None
    st = ctx.lib.sor_solve3d_f64(ctx.handle, pu, pb, pf, int(n), float(omega), float(tol),
                                 int(max_iters), int(check_every), _stream_handle(u),
                                 ctypes.byref(res), hbuf)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    h = list(hbuf[: res.iterations]) if hist else None
    return _result(st, res, h)


def residual_f64(u, boundary, rhs=None, r=None, ctx: Context | None = None):
    """Return (sum r^2, sum b^2, max|r|); fills r (n x n float64) if given."""
    import torch
    n = u.shape[0]
    pu = _check_tensor("u", u, torch.float64, (n, n))
    pb = _check_tensor("boundary", boundary, torch.float64, (4 * n,))
    pf = None if rhs is None else _check_tensor("rhs", rhs, torch.float64, (n, n))
    pr = None if r is None else _check_tensor("r", r, torch.float64, (n, n))
    ctx = ctx or context(u.device.index)
    stats = (ctypes.c_double * 3)()
    st = ctx.lib.sor_residual_f64(ctx.handle, pu, pb, pf, int(n), pr, stats,
                                  _stream_handle(u))
    ctx._check(st, (OK,))
    return float(stats[0]), float(stats[1]), float(stats[2])


def solve_mixed(u, boundary, rhs=None, omega=None, rel_tol=1e-10, max_outer=50,
                inner_bits=32, inner_iters=0, hist=False,
                ctx: Context | None = None) -> Result:
    """FP64 defect correction around FP32 or binary16-storage SOR, in place on u."""
    import torch
    n = u.shape[0]
    if omega is None:
        omega = omega_opt(n)
    pu = _check_tensor("u", u, torch.float64, (n, n))
    pb = _check_tensor("boundary", boundary, torch.float64, (4 * n,))
    pf = None if rhs is None else _check_tensor("rhs", rhs, torch.float64, (n, n))
    ctx = ctx or context(u.device.index)
    res = _Result()
    hbuf = (ctypes.c_double * (int(max_outer) + 1))() if hist else None
    st = ctx.lib.sor_solve_mixed(ctx.handle, pu, pb, pf, int(n), float(omega),
                                 float(rel_tol), int(max_outer), int(inner_bits),
                                 int(inner_iters), _stream_handle(u),
                                 ctypes.byref(res), hbuf)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    h = list(hbuf[: res.outer_steps + 1]) if hist else None
    return _result(st, res, h)


@dataclass
class MixedSpec:
    """One grid of a mixed-precision batched solve (torch float64 CUDA tensors)."""
    u: object
    boundary: object
    rhs: object = None
    omega: float | None = None
    rel_tol: float = 1e-10
    corr_tol: float = 0.0
    max_outer: int = 50
    inner_iters: int = 0


def batch_solve_mixed(specs, inner_bits=32, ctx: Context | None = None) -> list[Result]:
    """Mixed-precision defect correction for many grids in one persistent launch."""
    import torch
    specs = list(specs)
    if not specs:
        return []
    ctx = ctx or context(specs[0].u.device.index)
    descs = (_MixedDesc * len(specs))()
    for k, sp in enumerate(specs):
        n = sp.u.shape[0]
        d = descs[k]
        d.u = _check_tensor("u", sp.u, torch.float64, (n, n))
        d.boundary = _check_tensor("boundary", sp.boundary, torch.float64, (4 * n,))
        d.rhs = None if sp.rhs is None else _check_tensor("rhs", sp.rhs, torch.float64, (n, n))
        d.n = n
        d.omega = omega_opt(n) if sp.omega is None else sp.omega
        d.rel_tol = sp.rel_tol
        d.corr_tol = sp.corr_tol
        d.max_outer = sp.max_outer
        d.inner_iters = sp.inner_iters
    res = (_Result * len(specs))()
    st = ctx.lib.sor_batch_solve_mixed(ctx.handle, descs, len(specs), int(inner_bits),
                                       _stream_handle(specs[0].u), res)
    ctx._check(st, (OK, NOT_CONVERGED, ENONFINITE))
    return [_result(r.status, r) for r in res]


@dataclass
class Completion:
    ticket: int
    status: int
    result: Result
    submit_s: float
    admit_s: float
    done_s: float
    u: object                 # numpy n x n result


class Server:
    """Request loop of mixed-precision solves on one GPU (continuous batching).

    Requests carry host (numpy) arrays; results come back as numpy arrays."""

    def __init__(self, device=0, inner_bits=32, hbm_budget=8 << 30, max_slots=64,
                 slice_ms=2.0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.sor_server_create(int(device), int(inner_bits), int(hbm_budget),
                                        int(max_slots), float(slice_ms), ctypes.byref(h))
        if st != OK:
            raise SorError(st, "sor_server_create failed")
        self.handle = h
        self._n = {}

    def clock(self) -> float:
        return self.lib.sor_server_clock(self.handle)

    def submit(self, boundary, rhs=None, u0=None, omega=0.0, rel_tol=1e-8,
               corr_tol=0.0, max_outer=50, inner_iters=0) -> int:
        import numpy as np
        b = np.ascontiguousarray(boundary, dtype=np.float64)
        n = b.size // 4
        f = None if rhs is None else np.ascontiguousarray(rhs, dtype=np.float64).reshape(n, n)
        u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(n, n)
        r = _Request(None if u is None else u.ctypes.data, b.ctypes.data,
                     None if f is None else f.ctypes.data, n, 0, float(omega),
                     float(rel_tol), float(corr_tol), int(max_outer), int(inner_iters))
        t = ctypes.c_uint64()
        st = self.lib.sor_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t))
        if st != OK:
            raise SorError(st, "sor_server_submit failed")
        self._n[t.value] = n
        return t.value

    def poll(self, ticket, wait_ms=0.0):
        """Completion if the request finished, else None."""
        import numpy as np
        n = self._n[ticket]
        info = _RequestInfo()
        out = np.empty((n, n), dtype=np.float64)
        st = self.lib.sor_server_poll(self.handle, ctypes.c_uint64(ticket), float(wait_ms),
                                      ctypes.byref(info), out.ctypes.data)
        if st == EBUSY:
            return None
        if st == EINVAL:
            raise SorError(st, "unknown ticket")
        del self._n[ticket]
        return Completion(ticket, st, _result(st, info.result), info.submit_s,
                          info.admit_s, info.done_s, out)

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)]
        self.lib.sor_server_stats(self.handle, *[ctypes.byref(x) for x in v])
        return dict(launches=v[0].value, completed=v[1].value, waiting=v[2].value,
                    resident=v[3].value)

    def memory(self):
        """Device memory of request state: budget, bytes held now, most held."""
        v = [ctypes.c_size_t() for _ in range(3)]
        self.lib.sor_server_memory(self.handle, *[ctypes.byref(x) for x in v])
        return dict(budget=v[0].value, in_use=v[1].value, peak=v[2].value)

    def error(self) -> str:
        return self.lib.sor_server_last_error(self.handle).decode()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sor_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
