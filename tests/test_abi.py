"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point that include/sor.h declares, and reports its version."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sor.h")
LIB = os.path.join(ROOT, "paper_1401_0763_amd", "libsor.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sor_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for required in ("sor_ctx_create", "sor_ctx_destroy", "sor_last_error",
                     "sor_solve_f64", "sor_solve_f32", "sor_residual_f64",
                     "sor_solve_mixed", "sor_version"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libsor.so is not built"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sor_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_and_reports_version():
    lib = ctypes.CDLL(LIB)
    lib.sor_version.restype = ctypes.c_char_p
    assert lib.sor_version().decode().startswith("sor ")


def test_binding_loads_and_validates_without_gpu():
    import paper_1401_0763_amd as sor
    assert sor.version().endswith("gfx950")
    # a null context handle is rejected without touching a device
    lib = sor.load_library()
    t = sor._Tiling(4, 64)
    assert lib.sor_ctx_set_tiling(None, 64, ctypes.byref(t)) == sor.EINVAL
    assert lib.sor_solve_f64(None, None, None, None, 8, 1.5, 1e-6, 10, 1, None,
                             None, None) == sor.EINVAL


def test_newer_entry_points_reject_a_null_context():
    import paper_1401_0763_amd as sor
    lib = sor.load_library()
    assert lib.sor_solve3d_f64(None, None, None, None, 8, 1.5, 1e-6, 10, 1, None,
                               None, None) == sor.EINVAL
    assert lib.sor_solve_variant_f64(None, 1, None, None, None, 8, 1.0, 1e-6, 10, 1,
                                     None, None, None) == sor.EINVAL
    assert lib.sor_solve_blockpar_f64(None, None, None, None, 8, 1.0, 4, 4, 1e-6, 10, 1,
                                      None, None, None) == sor.EINVAL
    assert lib.sor_ctx_set_tiling3d(None, 0, 0, 0, 0) == sor.EINVAL
    tl = sor._Tiling(4, 64)
    assert lib.sor_ctx_set_variant_tiling(None, sor.ORDER_FOUR_COLOUR,
                                          ctypes.byref(tl)) == sor.EINVAL
    assert lib.sor_ctx_get_variant_tiling(None, sor.ORDER_FOUR_COLOUR,
                                          ctypes.byref(tl)) == sor.EINVAL
    t, a, b, c = (ctypes.c_int32() for _ in range(4))
    assert lib.sor_ctx_tiling3d_for(None, 64, 0, 10, ctypes.byref(t), ctypes.byref(a),
                                    ctypes.byref(b), ctypes.byref(c)) == sor.EINVAL


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with the shared library absent the binding raises."""
    import paper_1401_0763_amd as sor
    monkeypatch.setattr(sor, "LIB_PATH", str(tmp_path / "libsor.so"))
    monkeypatch.setattr(sor, "_lib", None)
    with pytest.raises(ImportError):
        sor.load_library()
    with pytest.raises(ImportError):
        sor.version()


def test_omega_opt_host_function():
    """sor_omega_opt is a host function (no device access): Young's optimum
    2 / (1 + sin(pi/(n+1))) as the library uses it where no omega is given."""
    import ctypes
    import math
    lib = ctypes.CDLL(LIB)
    lib.sor_omega_opt.restype = ctypes.c_double
    lib.sor_omega_opt.argtypes = [ctypes.c_int32]
    for n in (1, 2, 16, 32, 256, 4096, 65536):
        assert lib.sor_omega_opt(n) == 2.0 / (1.0 + math.sin(math.pi / (n + 1)))
    assert math.isnan(lib.sor_omega_opt(0))
    # the closed form of the survey's table (n = 256 and 4096)
    assert abs(lib.sor_omega_opt(256) - 1.975847650301681) < 1e-15
    assert abs(lib.sor_omega_opt(4096) - 1.998467568850995) < 1e-15


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: --gpus above 1 exits with status 2 and
    a message, before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
