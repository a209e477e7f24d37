"""CPU-only checks of the C ABI: the library loads, exports everything the
public header declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import errno
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exact.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exact_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2503_19925_amd import build, exact
    if not os.path.exists(exact.LIB_PATH):
        build.build()
    return exact.load()


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("exact_geometry_create", "exact_geometry_destroy", "exact_forward",
              "exact_backproject", "exact_operator", "exact_solve", "exact_step_size",
              "exact_last_error", "exact_solve_opts_default"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2503_19925_amd import exact
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(exact.EXPORTS) == set(declared_functions())


def test_opts_defaults(lib):
    from paper_2503_19925_amd.exact import SolveOpts
    o = SolveOpts()
    lib.exact_solve_opts_default(C.byref(o))
    assert o.gamma == 0.0 and o.gamma_scale == 0.25 and o.max_iters == 500
    assert o.tol == 0.0 and o.stop_mode == 0 and o.check_every == 16 and o.power_iters == 100
    assert o.lambda_hat == 0.0


def test_negative_lambda_hat_rejected(lib):
    """A given lambda_max must be finite and >= 0 (checked before any device
    work: the geometry handle is not even looked at first)."""
    from paper_2503_19925_amd.exact import SolveOpts
    o = SolveOpts()
    lib.exact_solve_opts_default(C.byref(o))
    for bad in (-1.0, float("nan"), float("inf")):
        o.lambda_hat = bad
        assert lib.exact_dense_solve(4, 2, C.c_void_p(16), None, None, C.c_void_p(16),
                                     C.byref(o), 0.0, None, None) == -errno.EINVAL
        assert "lambda_hat" in lib.exact_last_error().decode()


@pytest.mark.parametrize("args", [
    (0, 10, 10, 1, 0.1, 0.1),          # no pixels
    (16, 0, 10, 1, 0.1, 0.1),          # no views
    (16, 10, 0, 1, 0.1, 0.1),          # no bins
    (16, 10, 10, 3, 0.1, 0.1),         # neither 180 nor 360 degrees
    (16, 10, 10, 1, 0.0, 0.1),         # zero pixel size
    (16, 10, 10, 1, 0.1, float("nan")),
    (20000, 10, 10, 1, 0.1, 0.1),      # image too large
    (16, 65536, 65536, 1, 0.1, 0.1),   # too many rays
    (16, 32768, 32765, 1, 0.1, 0.1),   # padded sinogram past 32-bit byte offsets
])
def test_geometry_create_rejects(lib, args):
    h = C.c_void_p()
    assert lib.exact_geometry_create(*args, C.byref(h)) == -errno.EINVAL
    assert not h.value
    assert lib.exact_last_error().decode()


def test_null_handles_rejected(lib):
    assert lib.exact_forward(None, None, None, None) == -errno.EINVAL
    assert lib.exact_backproject(None, None, None, None) == -errno.EINVAL
    assert lib.exact_operator(None, None, None, None, None, None, None) == -errno.EINVAL
    assert lib.exact_solve(None, None, None, None, None, None, None) == -errno.EINVAL
    lam = C.c_double()
    assert lib.exact_step_size(None, None, 10, 0.25, C.byref(lam), None, None) == -errno.EINVAL
    assert lib.exact_geometry_destroy(None) == 0
    assert "NULL" in lib.exact_last_error().decode() or lib.exact_last_error() == b""


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2503_19925_amd import exact
    monkeypatch.setattr(exact, "_LIB", None)
    monkeypatch.setattr(exact, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        exact.load()


def test_run_footprint_is_host_arithmetic(lib):
    from paper_2503_19925_amd import exact
    # the counts, the padded residual (two zero bins at each end of a row),
    # four padded images (four zero columns at each end of a row, and a
    # tail of 64 zero floats) and small tables
    N, V, B = 512, 180, 725
    base = 4 * (V * B + V * (B + 4) + 4 * (N * (N + 8) + 64))
    f = exact.exact_run_footprint(N, V, B)
    assert base < f < base + 65536
    assert exact.exact_run_footprint(0, 10, 10) == 0


def test_batch_null_handles(lib):
    assert lib.exact_batch_step(None, 1, None) == -errno.EINVAL
    assert lib.exact_batch_sync(None) == -errno.EINVAL
    assert lib.exact_batch_poll(None, 0, None) == -errno.EINVAL
    assert lib.exact_batch_remove(None, 0) == -errno.EINVAL
    assert lib.exact_batch_destroy(None) == 0
    h = C.c_void_p()
    assert lib.exact_batch_create(1 << 20, 0, C.byref(h)) == -errno.EINVAL


def test_averaged_rule_is_exact_solve_only(lib):
    """The resident solver and the batch keep one live iterate and no ring of
    past iterates: they refuse the averaged-iterate stop rule."""
    from paper_2503_19925_amd.exact import SolveOpts, STOP_AVERAGED_ITERATE
    o = SolveOpts()
    lib.exact_solve_opts_default(C.byref(o))
    o.stop_mode = STOP_AVERAGED_ITERATE
    h = C.c_void_p()
    assert lib.exact_solver_create(None, None, None, None, C.byref(o), C.byref(h), None) == -errno.EINVAL
    assert "averaged" in lib.exact_last_error().decode()
    o.stop_mode = 7
    assert lib.exact_solve(None, None, None, None, C.byref(o), None, None) == -errno.EINVAL


def test_solver_profile_rejects_bad_arguments(lib):
    import ctypes
    out = (ctypes.c_double * 5)()
    assert lib.exact_solver_profile(None, 3, out, None) == -errno.EINVAL
    assert lib.exact_solver_time_kernels(None, 3, out, None) == -errno.EINVAL


def test_tv_entry_points_reject_bad_arguments(lib):
    from paper_2503_19925_amd.exact import TvOpts
    o = TvOpts()
    lib.exact_tv_opts_default(C.byref(o))
    assert (o.tv_tol, o.prox_iters, o.max_bisect, o.dyk_tol, o.max_outer) == (0.01, 100, 40, 1e-4, 200)
    out = C.c_double()
    assert lib.exact_tv_norm(0, None, C.byref(out), None) == -errno.EINVAL
    assert lib.exact_tv_norm(8, None, C.byref(out), None) == -errno.EINVAL
    assert lib.exact_tv_prox(8, None, 1.0, 10, None, None) == -errno.EINVAL
    assert lib.exact_project_tv(8, None, 1.0, None, None, None, None) == -errno.EINVAL
    fake = C.c_void_p(16)
    assert lib.exact_project_tv(8, fake, -1.0, None, fake, None, None) == -errno.EINVAL
    assert "tau" in lib.exact_last_error().decode()
    o.prox_iters = 0
    assert lib.exact_project_tv(8, fake, 1.0, C.byref(o), fake, None, None) == -errno.EINVAL
    assert lib.exact_solve_tv(None, None, None, None, None, 0.0, None, None, None, None) == -errno.EINVAL



def test_dense_entry_points_reject_bad_arguments(lib):
    from paper_2503_19925_amd.exact import Spectrum
    import numpy as np
    mu = np.array([1.0])
    w = np.array([1.0])
    sp = Spectrum(1, 1, mu.ctypes.data_as(C.POINTER(C.c_double)),
                  w.ctypes.data_as(C.POINTER(C.c_double)), None)
    fake = C.c_void_p(16)
    assert lib.exact_dense_operator(10, 5, None, C.byref(sp), fake, fake, fake, None) == -errno.EINVAL
    assert lib.exact_dense_solve(10, 5, fake, C.byref(sp), fake, None, None, 0.0, None, None) == -errno.EINVAL
    assert lib.exact_dense_solve(10, 5, fake, C.byref(sp), fake, fake, None, float("inf"), None,
                                 None) == -errno.EINVAL
