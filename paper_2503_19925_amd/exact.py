"""Python binding of libexact (include/exact.h): argument marshalling only.

Every computation happens in the HIP library; torch supplies device memory
and the current stream.  The module fails loudly if the compiled library is
missing: there is no fallback path.

Functions keep the C names:

    g = exact_geometry_create(n_pix, n_views, n_bins, pixel_cm, bin_cm, half_turns=1)
    exact_forward(g, x, s)              s = A x
    exact_backproject(g, r, img)        img = A^T r
    exact_operator(g, mu, weight, y, x, F, r=None)
    lam, gamma = exact_step_size(g, mu, weight, max_iters=100, gamma_scale=0.25)
    info = exact_solve(g, mu, weight, y, x, **opts)
    exact_geometry_destroy(g)

Tensors are float32 CUDA (HIP) tensors, contiguous, with the layouts of
include/exact.h: images [N*N] (or [N, N]), sinograms [V*B], counts
[Wn*V*B].  mu and weight are host float64 arrays ([K], [Wn*K]).
"""
import ctypes as C
import errno
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexact.so")
_LIB = None

EXACT_ENOTCONV = 1

EXPORTS = ("exact_solve_opts_default", "exact_last_error", "exact_geometry_create",
           "exact_geometry_destroy", "exact_forward", "exact_backproject",
           "exact_operator", "exact_operator_noalloc", "exact_step_size", "exact_solve", "exact_solver_create",
           "exact_solver_step", "exact_solver_poll", "exact_solver_destroy",
           "exact_solver_profile", "exact_solver_time_kernels", "exact_tv_opts_default", "exact_tv_norm", "exact_tv_prox",
           "exact_project_tv", "exact_solve_tv", "exact_dense_operator", "exact_dense_solve",
           "exact_count_nonzeros", "exact_run_footprint", "exact_batch_create",
           "exact_batch_add", "exact_batch_step", "exact_batch_sync", "exact_batch_poll",
           "exact_batch_remove", "exact_batch_destroy")

# exact_batch_poll results
RUNNING, FINISHED, CAPPED = 0, 1, 2
STOP_NATURAL_RESIDUAL, STOP_AVERAGED_ITERATE = 0, 1
# phases of exact_solver_profile
STEP_PHASES = 5
PHASE_NAMES = ("forward_residual_x", "back_update_half", "forward_residual_xh",
               "back_update_full", "finish")


class ExactError(RuntimeError):
    """A libexact call returned an error code."""

    def __init__(self, fn, code, msg):
        name = errno.errorcode.get(-code, str(code)) if code < 0 else str(code)
        super().__init__("%s failed (%s): %s" % (fn, name, msg))
        self.code = code


class Spectrum(C.Structure):
    _fields_ = [("n_energies", C.c_int32), ("n_windows", C.c_int32),
                ("mu", C.POINTER(C.c_double)), ("weight", C.POINTER(C.c_double)),
                ("background", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("gamma", C.c_double), ("gamma_scale", C.c_double),
                ("max_iters", C.c_int32), ("tol", C.c_double), ("stop_mode", C.c_int32),
                ("check_every", C.c_int32), ("power_iters", C.c_int32),
                ("lambda_hat", C.c_double)]


class TvOpts(C.Structure):
    _fields_ = [("tv_tol", C.c_double), ("prox_iters", C.c_int32), ("max_bisect", C.c_int32),
                ("dyk_tol", C.c_double), ("max_outer", C.c_int32)]


class TvInfo(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("solves", C.c_int32), ("tv", C.c_double),
                ("ms", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("resid", C.c_double), ("gamma", C.c_double),
                ("lambda_hat", C.c_double), ("ms", C.c_double)]


def load():
    """Loads libexact.so (built by paper_2503_19925_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError("libexact.so is not built (%s); run "
                          "`python -m paper_2503_19925_amd.build`" % LIB_PATH)
    # torch first: the library then binds to the HIP runtime torch loaded.
    # Loaded the other way round, the process holds two HIP runtimes and
    # torch finds no GPU.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "exact_solve_opts_default": ([C.POINTER(SolveOpts)], None),
        "exact_last_error": ([], C.c_char_p),
        "exact_geometry_create": ([i32, i32, i32, i32, dbl, dbl, C.POINTER(vp)], C.c_int),
        "exact_geometry_destroy": ([vp], C.c_int),
        "exact_forward": ([vp, vp, vp, vp], C.c_int),
        "exact_backproject": ([vp, vp, vp, vp], C.c_int),
        "exact_operator": ([vp, C.POINTER(Spectrum), vp, vp, vp, vp, vp], C.c_int),
        "exact_operator_noalloc": ([vp, C.POINTER(Spectrum), vp, vp, vp, vp, vp], C.c_int),
        "exact_step_size": ([vp, C.POINTER(Spectrum), i32, dbl, C.POINTER(dbl),
                             C.POINTER(dbl), vp], C.c_int),
        "exact_solve": ([vp, C.POINTER(Spectrum), vp, vp, C.POINTER(SolveOpts),
                         C.POINTER(SolveInfo), vp], C.c_int),
        "exact_solver_create": ([vp, C.POINTER(Spectrum), vp, vp, C.POINTER(SolveOpts),
                                 C.POINTER(vp), vp], C.c_int),
        "exact_solver_step": ([vp, i32, vp], C.c_int),
        "exact_solver_poll": ([vp, C.POINTER(SolveInfo)], C.c_int),
        "exact_solver_destroy": ([vp], C.c_int),
        "exact_solver_profile": ([vp, C.c_int32, C.POINTER(C.c_double), vp], C.c_int),
        "exact_solver_time_kernels": ([vp, C.c_int32, C.POINTER(C.c_double), vp], C.c_int),
        "exact_count_nonzeros": ([vp, C.POINTER(C.c_int64), vp], C.c_int),
        "exact_run_footprint": ([i32, i32, i32], C.c_size_t),
        "exact_batch_create": ([C.c_size_t, i32, C.POINTER(vp)], C.c_int),
        "exact_batch_add": ([vp, vp, C.POINTER(Spectrum), vp, vp, C.POINTER(SolveOpts),
                             C.POINTER(i32), vp], C.c_int),
        "exact_batch_step": ([vp, i32, vp], C.c_int),
        "exact_batch_sync": ([vp], C.c_int),
        "exact_batch_poll": ([vp, i32, C.POINTER(SolveInfo)], C.c_int),
        "exact_batch_remove": ([vp, i32], C.c_int),
        "exact_batch_destroy": ([vp], C.c_int),
        "exact_dense_operator": ([i32, i32, vp, C.POINTER(Spectrum), vp, vp, vp, vp], C.c_int),
        "exact_dense_solve": ([i32, i32, vp, C.POINTER(Spectrum), vp, vp, C.POINTER(SolveOpts), dbl,
                               C.POINTER(SolveInfo), vp], C.c_int),
        "exact_tv_opts_default": ([C.POINTER(TvOpts)], None),
        "exact_tv_norm": ([i32, vp, C.POINTER(dbl), vp], C.c_int),
        "exact_tv_prox": ([i32, vp, dbl, i32, vp, vp], C.c_int),
        "exact_project_tv": ([i32, vp, dbl, C.POINTER(TvOpts), vp, C.POINTER(TvInfo), vp],
                             C.c_int),
        "exact_solve_tv": ([vp, C.POINTER(Spectrum), vp, vp, C.POINTER(SolveOpts), dbl,
                            C.POINTER(TvOpts), C.POINTER(SolveInfo), C.POINTER(TvInfo), vp],
                           C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIB = lib
    return lib


def _check(fn, code):
    if code < 0:
        raise ExactError(fn, code, load().exact_last_error().decode())
    return code


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("%s must be contiguous float32" % name)
    if t.numel() != numel:
        raise ValueError("%s must hold %d values, has %d" % (name, numel, t.numel()))
    return C.c_void_p(t.data_ptr())


class Geometry:
    """Owns an exact_geometry handle."""

    def __init__(self, n_pix, n_views, n_bins, pixel_cm=None, bin_cm=None, half_turns=1):
        self.n_pix, self.n_views, self.n_bins = int(n_pix), int(n_views), int(n_bins)
        self.pixel_cm = 10.0 / self.n_pix if pixel_cm is None else float(pixel_cm)
        self.bin_cm = self.pixel_cm if bin_cm is None else float(bin_cm)
        self.half_turns = int(half_turns)
        h = C.c_void_p()
        _check("exact_geometry_create", load().exact_geometry_create(
            self.n_pix, self.n_views, self.n_bins, self.half_turns, self.pixel_cm,
            self.bin_cm, C.byref(h)))
        self.handle = h

    @property
    def d(self):
        return self.n_pix * self.n_pix

    @property
    def n(self):
        return self.n_views * self.n_bins

    def close(self):
        if self.handle is not None and self.handle.value:
            _check("exact_geometry_destroy", load().exact_geometry_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Spec:
    """Keeps the host arrays alive while a call uses them.  background: an
    optional float32 device tensor [V*B] of known materials' line
    integrals."""

    def __init__(self, mu, weight, background=None, n=None):
        self.mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).ravel())
        self.w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64).ravel())
        K = self.mu.size
        Wn = self.w.size // K if K else 0
        if K == 0 or Wn * K != self.w.size:
            raise ValueError("weight must hold n_windows * n_energies values")
        self.K, self.Wn = K, Wn
        self.bg = background
        bgp = _dev(background, n, "background") if background is not None else None
        self.s = Spectrum(K, Wn, self.mu.ctypes.data_as(C.POINTER(C.c_double)),
                          self.w.ctypes.data_as(C.POINTER(C.c_double)), bgp)


def exact_geometry_create(n_pix, n_views, n_bins, pixel_cm=None, bin_cm=None, half_turns=1):
    return Geometry(n_pix, n_views, n_bins, pixel_cm, bin_cm, half_turns)


def exact_geometry_destroy(g):
    g.close()


def exact_forward(g, x, s, stream=None):
    _check("exact_forward", load().exact_forward(
        g.handle, _dev(x, g.d, "x"), _dev(s, g.n, "s"), _stream(stream)))
    return s


def exact_backproject(g, r, img, stream=None):
    _check("exact_backproject", load().exact_backproject(
        g.handle, _dev(r, g.n, "r"), _dev(img, g.d, "img"), _stream(stream)))
    return img


def exact_operator(g, mu, weight, y, x, F, r=None, stream=None, background=None):
    sp = _Spec(mu, weight, background, g.n)
    _check("exact_operator", load().exact_operator(
        g.handle, C.byref(sp.s), _dev(y, sp.Wn * g.n, "y"), _dev(x, g.d, "x"),
        _dev(F, g.d, "F"), None if r is None else _dev(r, g.n, "r"), _stream(stream)))
    return F


def exact_operator_noalloc(g, mu, weight, y, x, F, r=None, stream=None, background=None):
    """exact_operator with its scratch in the library's static device array
    (no device allocation in the call); calls on one GPU must not overlap."""
    sp = _Spec(mu, weight, background, g.n)
    _check("exact_operator_noalloc", load().exact_operator_noalloc(
        g.handle, C.byref(sp.s), _dev(y, sp.Wn * g.n, "y"), _dev(x, g.d, "x"),
        _dev(F, g.d, "F"), None if r is None else _dev(r, g.n, "r"), _stream(stream)))
    return F


def exact_step_size(g, mu=None, weight=None, max_iters=100, gamma_scale=0.25, stream=None):
    sp = _Spec(mu, weight) if mu is not None else None
    lam, gam = C.c_double(), C.c_double()
    _check("exact_step_size", load().exact_step_size(
        g.handle, C.byref(sp.s) if sp else None, int(max_iters), float(gamma_scale),
        C.byref(lam), C.byref(gam), _stream(stream)))
    return lam.value, gam.value


def _opts(gamma, gamma_scale, max_iters, tol, check_every, power_iters,
          stop_mode=STOP_NATURAL_RESIDUAL, lambda_hat=0.0):
    o = SolveOpts()
    load().exact_solve_opts_default(C.byref(o))
    o.gamma, o.gamma_scale, o.max_iters, o.tol = float(gamma), float(gamma_scale), int(max_iters), float(tol)
    o.check_every, o.power_iters = int(check_every), int(power_iters)
    o.stop_mode = int(stop_mode)
    o.lambda_hat = float(lambda_hat)
    return o


def _info_dict(info):
    return dict(iters=info.iters, resid=info.resid, gamma=info.gamma,
                lambda_hat=info.lambda_hat, ms=info.ms)


def exact_count_nonzeros(g, stream=None):
    out = C.c_int64()
    _check("exact_count_nonzeros", load().exact_count_nonzeros(g.handle, C.byref(out), _stream(stream)))
    return out.value


class Solver:
    """A resident run (exact_solver_*): state stays on the device and
    step(n) enqueues n full extragradient steps on the stream."""

    def __init__(self, g, mu, weight, y, x, gamma=0.0, gamma_scale=0.25, max_iters=500, tol=0.0,
                 check_every=16, power_iters=100, stream=None, background=None, lambda_hat=0.0):
        sp = _Spec(mu, weight, background, g.n)
        self.g, self.x = g, x
        o = _opts(gamma, gamma_scale, max_iters, tol, check_every, power_iters,
                  lambda_hat=lambda_hat)
        h = C.c_void_p()
        _check("exact_solver_create", load().exact_solver_create(
            g.handle, C.byref(sp.s), _dev(y, sp.Wn * g.n, "y"), _dev(x, g.d, "x"), C.byref(o),
            C.byref(h), _stream(stream)))
        self.handle = h

    def step(self, n_steps=1, stream=None):
        _check("exact_solver_step", load().exact_solver_step(self.handle, int(n_steps), _stream(stream)))

    def poll(self):
        """(done, info dict); waits for the enqueued steps."""
        info = SolveInfo()
        done = _check("exact_solver_poll", load().exact_solver_poll(self.handle, C.byref(info)))
        return bool(done), _info_dict(info)

    def profile(self, n_steps, stream=None):
        """Runs n_steps more steps kernel by kernel with HIP events around
        each phase; returns the average ms of the STEP_PHASES phases."""
        out = (C.c_double * STEP_PHASES)()
        _check("exact_solver_profile", load().exact_solver_profile(
            self.handle, int(n_steps), out, _stream(stream)))
        return list(out)

    def time_kernels(self, reps, stream=None):
        """Average ms per launch of each of the STEP_PHASES phase kernels,
        each launched reps times back to back between two HIP events; the
        run's state is left as it was."""
        out = (C.c_double * STEP_PHASES)()
        _check("exact_solver_time_kernels", load().exact_solver_time_kernels(
            self.handle, int(reps), out, _stream(stream)))
        return list(out)

    def close(self):
        if self.handle is not None and self.handle.value:
            _check("exact_solver_destroy", load().exact_solver_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exact_solve(g, mu, weight, y, x, gamma=0.0, gamma_scale=0.25, max_iters=500, tol=0.0,
                check_every=16, power_iters=100, stream=None, stop_mode=STOP_NATURAL_RESIDUAL,
                background=None, lambda_hat=0.0):
    """Runs EXACT in place on x.  Returns a dict with iters, resid, gamma,
    lambda_hat, ms and converged (True/False, or None when tol == 0).  With
    stop_mode=STOP_AVERAGED_ITERATE x receives the averaged iterate and tol
    bounds ||xbar_{t+1} - xbar_t|| (absolute).  background: known materials'
    line integrals per ray (device float32 [V*B]) or None.  lambda_hat > 0:
    the geometry's lambda_max, known already, for the automatic step size."""
    sp = _Spec(mu, weight, background, g.n)
    o = _opts(gamma, gamma_scale, max_iters, tol, check_every, power_iters, stop_mode,
              lambda_hat=lambda_hat)
    info = SolveInfo()
    code = _check("exact_solve", load().exact_solve(
        g.handle, C.byref(sp.s), _dev(y, sp.Wn * g.n, "y"), _dev(x, g.d, "x"), C.byref(o),
        C.byref(info), _stream(stream)))
    d = _info_dict(info)
    d["converged"] = (code == 0) if tol > 0 else None
    return d


def exact_run_footprint(n_pix, n_views, n_bins):
    """Device bytes the library allocates for one run (x and y not included)."""
    return int(load().exact_run_footprint(int(n_pix), int(n_views), int(n_bins)))


class Batch:
    """exact_batch_*: many runs of different shapes advanced together.

    add() returns a slot; step(n) enqueues n steps of every run; sync()
    waits and returns how many runs are still running; poll(slot) gives
    (status, info) with status RUNNING, FINISHED or CAPPED."""

    def __init__(self, hbm_budget_bytes, capacity=256):
        h = C.c_void_p()
        _check("exact_batch_create", load().exact_batch_create(
            C.c_size_t(int(hbm_budget_bytes)), int(capacity), C.byref(h)))
        self.handle = h
        self._keep = {}

    def add(self, g, mu, weight, y, x, gamma=0.0, gamma_scale=0.25, max_iters=500, tol=0.0,
            power_iters=100, stream=None, background=None, lambda_hat=0.0):
        sp = _Spec(mu, weight, background, g.n)
        o = _opts(gamma, gamma_scale, max_iters, tol, 1, power_iters, lambda_hat=lambda_hat)
        slot = C.c_int32(-1)
        _check("exact_batch_add", load().exact_batch_add(
            self.handle, g.handle, C.byref(sp.s), _dev(y, sp.Wn * g.n, "y"), _dev(x, g.d, "x"),
            C.byref(o), C.byref(slot), _stream(stream)))
        self._keep[slot.value] = (g, x)
        return slot.value

    def step(self, n_steps=1, stream=None):
        _check("exact_batch_step", load().exact_batch_step(self.handle, int(n_steps), _stream(stream)))

    def sync(self):
        return _check("exact_batch_sync", load().exact_batch_sync(self.handle))

    def poll(self, slot):
        info = SolveInfo()
        st = _check("exact_batch_poll", load().exact_batch_poll(self.handle, int(slot), C.byref(info)))
        return st, _info_dict(info)

    def remove(self, slot):
        _check("exact_batch_remove", load().exact_batch_remove(self.handle, int(slot)))
        self._keep.pop(slot, None)

    def close(self):
        if self.handle is not None and self.handle.value:
            _check("exact_batch_destroy", load().exact_batch_destroy(self.handle))
        self.handle = None
        self._keep = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- TV ball

def _tv_opts(**kw):
    o = TvOpts()
    load().exact_tv_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown TV option %r" % k)
        setattr(o, k, v)
    return o


def _side(t):
    n = int(round(t.numel() ** 0.5))
    if n * n != t.numel():
        raise ValueError("image must be square")
    return n


def exact_tv_norm(x, stream=None):
    """Isotropic TV (forward differences) of a square device image."""
    n = _side(x)
    out = C.c_double()
    _check("exact_tv_norm", load().exact_tv_norm(n, _dev(x, n * n, "x"), C.byref(out),
                                                 _stream(stream)))
    return out.value


def exact_tv_prox(b, lam, x, iters=100, stream=None):
    """x = argmin ||x - b||^2 + lam TV(x) by `iters` FGP steps."""
    n = _side(b)
    _check("exact_tv_prox", load().exact_tv_prox(n, _dev(b, n * n, "b"), float(lam), int(iters),
                                                 _dev(x, n * n, "x"), _stream(stream)))
    return x


def _tv_info(i):
    return dict(rounds=i.rounds, solves=i.solves, tv=i.tv, ms=i.ms)


def exact_project_tv(z, tau, out, stream=None, **tvopts):
    """out = projection of z onto {TV <= tau} and the orthant (Dykstra).
    Returns a dict with rounds, solves, tv, ms."""
    n = _side(z)
    o = _tv_opts(**tvopts)
    info = TvInfo()
    _check("exact_project_tv", load().exact_project_tv(
        n, _dev(z, n * n, "z"), float(tau), C.byref(o), _dev(out, n * n, "out"), C.byref(info),
        _stream(stream)))
    return _tv_info(info)


def exact_solve_tv(g, mu, weight, y, x, tau, gamma=0.0, gamma_scale=0.25, max_iters=500,
                   tol=0.0, power_iters=100, stream=None, background=None, **tvopts):
    """EXACT over {TV <= tau} and the orthant, in place on x.  Returns
    (solve info dict with converged, TV info dict)."""
    sp = _Spec(mu, weight, background, g.n)
    o = _opts(gamma, gamma_scale, max_iters, tol, 16, power_iters)
    to = _tv_opts(**tvopts)
    info, tinfo = SolveInfo(), TvInfo()
    code = _check("exact_solve_tv", load().exact_solve_tv(
        g.handle, C.byref(sp.s), _dev(y, sp.Wn * g.n, "y"), _dev(x, g.d, "x"), C.byref(o),
        float(tau), C.byref(to), C.byref(info), C.byref(tinfo), _stream(stream)))
    d = _info_dict(info)
    d["converged"] = (code == 0) if tol > 0 else None
    return d, _tv_info(tinfo)


# ------------------------------------------------------- dense measurements

def _dense_shape(A):
    if A.dim() != 2:
        raise ValueError("A must be a 2-D device tensor (n x d)")
    return int(A.shape[0]), int(A.shape[1])


def exact_dense_operator(A, mu, weight, y, x, F, stream=None):
    """F = (1/n) A^T r for an explicit n x d matrix A (device, float32)."""
    n, d = _dense_shape(A)
    sp = _Spec(mu, weight)
    _check("exact_dense_operator", load().exact_dense_operator(
        n, d, _dev(A, n * d, "A"), C.byref(sp.s), _dev(y, sp.Wn * n, "y"), _dev(x, d, "x"),
        _dev(F, d, "F"), _stream(stream)))
    return F


def exact_dense_solve(A, mu, weight, y, x, gamma=0.0, gamma_scale=0.25, max_iters=500, tol=0.0,
                      radius=0.0, check_every=16, power_iters=100, stream=None):
    """EXACT with an explicit matrix over the ball of the given radius
    (radius <= 0: unconstrained), in place on x.  Returns the info dict."""
    n, d = _dense_shape(A)
    sp = _Spec(mu, weight)
    o = _opts(gamma, gamma_scale, max_iters, tol, check_every, power_iters)
    info = SolveInfo()
    code = _check("exact_dense_solve", load().exact_dense_solve(
        n, d, _dev(A, n * d, "A"), C.byref(sp.s), _dev(y, sp.Wn * n, "y"), _dev(x, d, "x"),
        C.byref(o), float(radius), C.byref(info), _stream(stream)))
    out = _info_dict(info)
    out["converged"] = (code == 0) if tol > 0 else None
    return out
