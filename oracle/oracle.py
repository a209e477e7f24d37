"""ctypes front end of the EXACT CPU oracle -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
module.  It loads oracle/liboracle.so (built by oracle/build.py) and exposes
numpy-in / numpy-out functions.  `prec` selects the arithmetic of the same C
source: "f64" (the oracle proper), "ld" (x87 long double, used to state the
oracle's own rounding error) or "f32" (single precision, used to measure how
sensitive a computation is to float rounding).

Conventions (shared with the C source, see exact_oracle.c):
  image x:      float64 [N*N], p = iy*N + ix, iy = 0 the bottom row
  sinogram:     float64 [V*B], ray i = v*B + b
  counts y:     float64 [Wn*V*B], window-major
  mu:           float64 [K] (cm^2/g);  I: float64 [Wn*K] = Ibar_j * s_jk
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_PRECS = ("f64", "ld", "f32")


class Geom(C.Structure):
    """Parallel-beam geometry: N x N pixels of side pixel_cm, V views over
    half_turns*180 degrees, B detector bins of width bin_cm."""

    _fields_ = [("n_pix", C.c_int), ("n_views", C.c_int), ("n_bins", C.c_int),
                ("half_turns", C.c_int), ("pixel_cm", C.c_double),
                ("bin_cm", C.c_double)]

    def __init__(self, n_pix, n_views, n_bins, pixel_cm=None, bin_cm=None,
                 half_turns=1):
        if pixel_cm is None:
            pixel_cm = 10.0 / n_pix
        if bin_cm is None:
            bin_cm = pixel_cm
        super().__init__(int(n_pix), int(n_views), int(n_bins), int(half_turns),
                         float(pixel_cm), float(bin_cm))

    @property
    def d(self):
        return self.n_pix * self.n_pix

    @property
    def n(self):
        return self.n_views * self.n_bins


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_gp = C.POINTER(Geom)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle.build import build as _build
            _build()
        _LIB = C.CDLL(path)
        for p in _PRECS:
            f = getattr(_LIB, "ora_forward_" + p)
            f.argtypes = [_gp, _dp, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_forward_rays_" + p)
            f.argtypes = [_gp, _dp, C.c_int, _lp, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_back_" + p)
            f.argtypes = [_gp, _dp, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_back_pixels_" + p)
            f.argtypes = [_gp, _dp, C.c_int, _lp, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_residual_" + p)
            f.argtypes = [C.c_long, C.c_int, C.c_int, _dp, _dp, _dp, _dp, C.c_void_p, _dp, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_operator_" + p)
            f.argtypes = [_gp, C.c_int, C.c_int, _dp, _dp, _dp, C.c_void_p, _dp, _dp,
                          C.c_void_p, C.c_void_p]
            f.restype = None
            f = getattr(_LIB, "ora_eg_" + p)
            f.argtypes = [_gp, C.c_int, C.c_int, _dp, _dp, _dp, C.c_void_p, _dp, C.c_double,
                          C.c_int, C.c_double, C.c_void_p]
            f.restype = C.c_int
            f = getattr(_LIB, "ora_eg_avg_" + p)
            f.argtypes = [_gp, C.c_int, C.c_int, _dp, _dp, _dp, C.c_void_p, _dp, C.c_double,
                          C.c_int, C.c_double, C.c_void_p, C.c_void_p]
            f.restype = C.c_int
            f = getattr(_LIB, "ora_window_mean_" + p)
            f.argtypes = [_dp, C.c_long, C.c_int, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_tv_norm_" + p)
            f.argtypes = [C.c_int, _dp]
            f.restype = C.c_double
            f = getattr(_LIB, "ora_tv_prox_" + p)
            f.argtypes = [C.c_int, _dp, C.c_double, C.c_int, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_tv_ball_" + p)
            f.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                          _dp, C.POINTER(C.c_double)]
            f.restype = C.c_int
            f = getattr(_LIB, "ora_project_tv_" + p)
            f.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                          C.c_int, _dp, C.POINTER(C.c_int)]
            f.restype = C.c_int
            f = getattr(_LIB, "ora_eg_tv_" + p)
            f.argtypes = [_gp, C.c_int, C.c_int, _dp, _dp, _dp, C.c_void_p, _dp, C.c_double,
                          C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                          C.c_double, C.c_int, C.c_void_p, C.POINTER(C.c_int)]
            f.restype = C.c_int
            f = getattr(_LIB, "ora_dense_operator_" + p)
            f.argtypes = [C.c_long, C.c_long, _dp, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
            f.restype = None
            f = getattr(_LIB, "ora_dense_eg_" + p)
            f.argtypes = [C.c_long, C.c_long, _dp, C.c_int, C.c_int, _dp, _dp, _dp, _dp,
                          C.c_double, C.c_double, C.c_int, C.c_double, C.c_void_p]
            f.restype = C.c_int
            f = getattr(_LIB, "ora_power_" + p)
            f.argtypes = [_gp, C.c_int, C.c_double, C.POINTER(C.c_int)]
            f.restype = C.c_double
            f = getattr(_LIB, "ora_nnz_" + p)
            f.argtypes = [_gp]
            f.restype = C.c_long
    return _LIB


def _fn(name, prec):
    if prec not in _PRECS:
        raise ValueError("prec must be one of %s" % (_PRECS,))
    return getattr(_lib(), "ora_%s_%s" % (name, prec))


def _f64(a, size=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
    if size is not None and a.size != size:
        raise ValueError("expected %d values, got %d" % (size, a.size))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def forward(g, x, prec="f64"):
    """s = A x (all rays)."""
    x = _f64(x, g.d)
    s = np.empty(g.n)
    _fn("forward", prec)(C.byref(g), x, s)
    return s


def forward_rays(g, x, rays, prec="f64"):
    """(A x)_i for the given ray indices only."""
    x = _f64(x, g.d)
    rays = np.ascontiguousarray(np.asarray(rays, dtype=np.int64).ravel())
    out = np.empty(rays.size)
    _fn("forward_rays", prec)(C.byref(g), x, int(rays.size), rays, out)
    return out


def back(g, r, prec="f64"):
    """A^T r (scatter form, no 1/n)."""
    r = _f64(r, g.n)
    img = np.empty(g.d)
    _fn("back", prec)(C.byref(g), r, img)
    return img


def back_pixels(g, r, pixels, prec="f64"):
    """(A^T r)_p for the given pixel indices, from the entry definition."""
    r = _f64(r, g.n)
    pixels = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64).ravel())
    out = np.empty(pixels.size)
    _fn("back_pixels", prec)(C.byref(g), r, int(pixels.size), pixels, out)
    return out


def _bg(bg, n):
    return None if bg is None else _f64(bg, n)


def residual(s, mu, I, y, prec="f64", bg=None):
    """Per-ray residual r = sum_j y_j - sum_j sum_k I_jk exp(-mu_k s_+);
    returns (r, model).  bg (optional, per ray): line integrals of known
    materials, entering through the reparametrised per-ray spectrum."""
    s = _f64(s)
    n = s.size
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    if Wn * K != I.size:
        raise ValueError("I must hold Wn*K values")
    y = _f64(y, Wn * n)
    r = np.empty(n)
    m = np.empty(n)
    b = _bg(bg, n)
    _fn("residual", prec)(n, K, Wn, mu, I, y, s, _ptr(b), r, m)
    return r, m


def operator(g, mu, I, y, x, prec="f64", want_sr=False, bg=None):
    """F(x) = (1/n) A^T r.  With want_sr also returns s = Ax and r."""
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    y = _f64(y, Wn * g.n)
    x = _f64(x, g.d)
    F = np.empty(g.d)
    s = np.empty(g.n) if want_sr else None
    r = np.empty(g.n) if want_sr else None
    b = _bg(bg, g.n)
    _fn("operator", prec)(C.byref(g), K, Wn, mu, I, y, _ptr(b), x, F, _ptr(s), _ptr(r))
    return (F, s, r) if want_sr else F


def eg(g, mu, I, y, x1, gamma, max_iters, tol=0.0, prec="f64", bg=None):
    """Projected extragradient from x1.  Returns (x_last, steps, rho_hist)."""
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    y = _f64(y, Wn * g.n)
    x = _f64(x1, g.d).copy()
    hist = np.full(max(int(max_iters), 1), np.nan)
    b = _bg(bg, g.n)
    t = _fn("eg", prec)(C.byref(g), K, Wn, mu, I, y, _ptr(b), x, float(gamma),
                        int(max_iters), float(tol), _ptr(hist))
    return x, int(t), hist[:t]


def eg_avg(g, mu, I, y, x1, gamma, max_iters, tol=0.0, prec="f64", bg=None):
    """Projected extragradient with the averaged-iterate stopping rule.
    Returns (xbar, steps, crit_hist, x_last): xbar at index steps+1, the
    history of ||xbar_{t+1} - xbar_t|| and the last iterate x_{steps+1}."""
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    y = _f64(y, Wn * g.n)
    x = _f64(x1, g.d).copy()
    last = np.empty(g.d)
    hist = np.full(max(int(max_iters), 1), np.nan)
    b = _bg(bg, g.n)
    t = _fn("eg_avg", prec)(C.byref(g), K, Wn, mu, I, y, _ptr(b), x, float(gamma),
                            int(max_iters), float(tol), _ptr(hist), _ptr(last))
    return x, int(t), hist[:t], last


def window_mean(traj, s, prec="f64"):
    """Mean of rows floor(s/2)+1 .. s (1-based) of traj [>= s, d]."""
    traj = np.ascontiguousarray(np.asarray(traj, dtype=np.float64))
    d = traj.shape[1]
    if traj.shape[0] < s or s < 1:
        raise ValueError("need 1 <= s <= rows")
    out = np.empty(d)
    _fn("window_mean", prec)(np.ascontiguousarray(traj[:s]).ravel(), d, int(s), out)
    return out


# TV-ball projection parameters: the paper's tolerances (|TV - tau| <= 0.01,
# Dykstra ||z_{k+1} - z_k|| <= 1e-4) and this implementation's fixed
# inner counts.
TV_DEFAULTS = dict(tv_tol=0.01, prox_iters=100, max_bisect=40, dyk_tol=1e-4, max_outer=200)


def _img(x, N=None):
    x = _f64(x)
    n = int(round(np.sqrt(x.size))) if N is None else int(N)
    if n * n != x.size:
        raise ValueError("image must be square")
    return x, n


def tv_norm(x, prec="f64"):
    """Isotropic TV (forward differences) of a square image."""
    x, N = _img(x)
    return float(_fn("tv_norm", prec)(N, x))


def tv_prox(b, lam, iters=TV_DEFAULTS["prox_iters"], prec="f64"):
    """argmin_x ||x - b||^2 + lam TV(x) by `iters` fast-gradient-projection
    steps on the dual, from zero."""
    b, N = _img(b)
    x = np.empty(N * N)
    _fn("tv_prox", prec)(N, b, float(lam), int(iters), x)
    return x


def tv_ball(v, tau, tv_tol=TV_DEFAULTS["tv_tol"], prox_iters=TV_DEFAULTS["prox_iters"],
            max_bisect=TV_DEFAULTS["max_bisect"], lam0=0.0, prec="f64"):
    """Approximate projection onto {TV <= tau} by binary search on the TV
    weight, cold (lam0 <= 0) or warm-started at lam0.  Returns (x, lam,
    proximal solves)."""
    v, N = _img(v)
    out = np.empty(N * N)
    lam = C.c_double(0.0)
    ns = _fn("tv_ball", prec)(N, v, float(tau), float(tv_tol), int(prox_iters),
                              int(max_bisect), float(lam0), out, C.byref(lam))
    return out, lam.value, int(ns)


def project_tv(z, tau, tv_tol=TV_DEFAULTS["tv_tol"], prox_iters=TV_DEFAULTS["prox_iters"],
               max_bisect=TV_DEFAULTS["max_bisect"], dyk_tol=TV_DEFAULTS["dyk_tol"],
               max_outer=TV_DEFAULTS["max_outer"], prec="f64"):
    """Projection onto {TV <= tau} intersected with x >= 0 by Dykstra's
    algorithm.  Returns (x, rounds, proximal solves)."""
    z, N = _img(z)
    out = np.empty(N * N)
    ns = C.c_int(0)
    k = _fn("project_tv", prec)(N, z, float(tau), float(tv_tol), int(prox_iters),
                                int(max_bisect), float(dyk_tol), int(max_outer), out,
                                C.byref(ns))
    return out, int(k), ns.value


def eg_tv(g, mu, I, y, x1, gamma, max_iters, tau, tol=0.0, prec="f64", bg=None,
          want_solves=False, **tvkw):
    """Projected extragradient over TV ball intersected with the orthant.
    Returns (x_last, steps, rho_hist); with want_solves=True also the
    number of TV-regularized points the run computed."""
    kw = dict(TV_DEFAULTS)
    kw.update(tvkw)
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    y = _f64(y, Wn * g.n)
    x = _f64(x1, g.d).copy()
    hist = np.full(max(int(max_iters), 1), np.nan)
    b = _bg(bg, g.n)
    ns = C.c_int(0)
    t = _fn("eg_tv", prec)(C.byref(g), K, Wn, mu, I, y, _ptr(b), x, float(gamma),
                           int(max_iters), float(tol), float(tau), float(kw["tv_tol"]),
                           int(kw["prox_iters"]), int(kw["max_bisect"]), float(kw["dyk_tol"]),
                           int(kw["max_outer"]), _ptr(hist), C.byref(ns))
    if want_solves:
        return x, int(t), hist[:t], ns.value
    return x, int(t), hist[:t]


def dense_operator(A, mu, I, y, x, prec="f64"):
    """F(x) = (1/n) A^T r for an explicit n x d matrix A (row-major)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n, d = A.shape
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    F = np.empty(d)
    _fn("dense_operator", prec)(n, d, A.ravel(), K, Wn, mu, I, _f64(y, Wn * n), _f64(x, d), F)
    return F


def dense_eg(A, mu, I, y, x1, gamma, max_iters, radius=0.0, tol=0.0, prec="f64"):
    """Projected extragradient with an explicit A over the ball of the given
    radius around 0 (radius <= 0: unconstrained).  Returns (x, steps, rho)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n, d = A.shape
    mu = _f64(mu)
    K = mu.size
    I = _f64(I)
    Wn = I.size // K
    x = _f64(x1, d).copy()
    hist = np.full(max(int(max_iters), 1), np.nan)
    t = _fn("dense_eg", prec)(n, d, A.ravel(), K, Wn, mu, I, _f64(y, Wn * n), x, float(gamma),
                              float(radius), int(max_iters), float(tol), _ptr(hist))
    return x, int(t), hist[:t]


def power(g, max_iters=10000, rel_tol=1e-12, prec="f64"):
    """lambda_max(A^T A / n) by power iteration.  Returns (lambda, iters)."""
    it = C.c_int(0)
    lam = _fn("power", prec)(C.byref(g), int(max_iters), float(rel_tol), C.byref(it))
    return lam, it.value


def nnz(g, prec="f64"):
    """Exact number of positive entries of A."""
    return int(_fn("nnz", prec)(C.byref(g)))


def step_size(lam, mu, I, c_gamma=0.25):
    """gamma = c / (lambda_max(Sigma) * sum_k J_k mu_k), J_k = sum_j I_jk
    (Theorem 2's step size with the multi-window Lipschitz bound)."""
    mu = np.asarray(mu, dtype=np.float64)
    J = np.asarray(I, dtype=np.float64).reshape(-1, mu.size).sum(axis=0)
    return c_gamma / (lam * float(np.dot(J, mu)))
