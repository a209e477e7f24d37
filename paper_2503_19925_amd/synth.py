"""Seeded synthetic inputs for EXACT reconstructions.

This module only *generates inputs*: random-ellipse phantoms, their exact
(analytic) line integrals, the energy spectrum and detector windows, and
Poisson photon counts drawn from the polychromatic measurement model.  It
holds none of the reconstruction's arithmetic (no discrete projector, no
operator, no iteration), so the CPU oracle and the HIP path can both be fed
from it without sharing any code with each other.

Measurement model simulated (paper Sec. 1, eq. model:multi-material with one
material, and the Poisson model of Sec. 1.2, eq. Poisson-model):

    y[j][i] ~ Poisson( sum_k I[j][k] exp(-mu_k * l_i) )

where l_i is the exact line integral of the continuous phantom along ray i,
I[j][k] = Ibar_j s_{jk} and the windows partition the energy bins.

Geometry conventions (the same definitions the library documents):
  * image: N x N pixels of side pixel_cm, centred at the origin; pixel
    (iy, ix) has centre ((ix-c) pixel_cm, (iy-c) pixel_cm), c = (N-1)/2;
  * view v at theta_v = half_turns * pi * v / V; detector bin b at
    u_b = (b - (B-1)/2) * bin_cm; ray i = v*B + b is the line
    {p : p . (cos theta_v, sin theta_v) = u_b}.

Choices the paper leaves open and this module fixes (all parameters):
  * energy bins: K equal bins over 20-120 keV, centres E_k = 20+(k+1/2)100/K;
  * source spectrum p_k proportional to E_k (120 - E_k), sum_k p_k = 1, so a
    ray receives I0 photons on average over all bins;
  * attenuation mu_k = 0.2 (40/E_k)^3 + 0.18 cm^2/g;
  * windows: Wn contiguous groups of bins with edges floor(j K / Wn) and unit
    sensitivity inside, so I[j][k] = I0 p_k for k in window j;
  * phantom: additive ellipses, centres uniform in a disc of radius 0.65 R,
    semi-axes uniform in [0.05 R, 0.30 R], orientation uniform in [0, pi),
    density uniform in [0.2, 1.5] g/cm^3, R = 5 cm (half the 10 cm field);
  * reference pixels (for RMSE only): 4 x 4 supersampled area averages.
"""
from dataclasses import dataclass, field
import math

import numpy as np

FOV_CM = 10.0


# ------------------------------------------------------------------ spectrum

def spectrum(K, Wn, I0):
    """Returns (mu[K], I[Wn*K]) as float64; I is window-major."""
    K, Wn = int(K), int(Wn)
    if K < 1 or Wn < 1 or Wn > K:
        raise ValueError("need 1 <= Wn <= K")
    E = 20.0 + (np.arange(K) + 0.5) * 100.0 / K
    p = E * (120.0 - E)
    p = p / p.sum()
    mu = 0.2 * (40.0 / E) ** 3 + 0.18
    I = np.zeros((Wn, K))
    for j in range(Wn):
        lo, hi = (j * K) // Wn, ((j + 1) * K) // Wn
        I[j, lo:hi] = I0 * p[lo:hi]
    return mu, I.ravel()


# ------------------------------------------------------------------- phantom

def ellipses(n_ell, seed, radius_cm=FOV_CM / 2):
    """Random ellipses as an array of rows (cx, cy, a, b, phi, rho)."""
    rng = np.random.default_rng(int(seed))
    R = float(radius_cm)
    rc = 0.65 * R * np.sqrt(rng.uniform(0.0, 1.0, n_ell))
    ac = rng.uniform(0.0, 2.0 * math.pi, n_ell)
    a = rng.uniform(0.05 * R, 0.30 * R, n_ell)
    b = rng.uniform(0.05 * R, 0.30 * R, n_ell)
    phi = rng.uniform(0.0, math.pi, n_ell)
    rho = rng.uniform(0.2, 1.5, n_ell)
    return np.stack([rc * np.cos(ac), rc * np.sin(ac), a, b, phi, rho], axis=1)


def phantom_image(ell, n_pix, pixel_cm=None, supersample=4):
    """Pixel averages of the continuous phantom (float64 [N*N])."""
    N = int(n_pix)
    if pixel_cm is None:
        pixel_cm = FOV_CM / N
    S = int(supersample)
    c = (N - 1) / 2.0
    img = np.zeros((N, N))
    sub = (np.arange(S) + 0.5) / S - 0.5          # sub-pixel offsets
    for cx, cy, a, b, phi, rho in ell:
        ext = max(a, b) / pixel_cm + 1.0
        ix0 = max(int(math.floor(cx / pixel_cm + c - ext)), 0)
        ix1 = min(int(math.ceil(cx / pixel_cm + c + ext)), N - 1)
        iy0 = max(int(math.floor(cy / pixel_cm + c - ext)), 0)
        iy1 = min(int(math.ceil(cy / pixel_cm + c + ext)), N - 1)
        if ix1 < ix0 or iy1 < iy0:
            continue
        ix = np.arange(ix0, ix1 + 1)
        iy = np.arange(iy0, iy1 + 1)
        X = ((ix[None, :, None, None] - c) + sub[None, None, None, :]) * pixel_cm
        Y = ((iy[:, None, None, None] - c) + sub[None, None, :, None]) * pixel_cm
        dx, dy = X - cx, Y - cy
        cp, sp = math.cos(phi), math.sin(phi)
        q = ((dx * cp + dy * sp) / a) ** 2 + ((-dx * sp + dy * cp) / b) ** 2
        inside = (q <= 1.0).mean(axis=(2, 3))
        img[iy0:iy1 + 1, ix0:ix1 + 1] += rho * inside
    return img.ravel()


def analytic_sinogram(ell, n_views, n_bins, bin_cm, half_turns=1):
    """Exact line integrals (g/cm^2) of the ellipse phantom, float64 [V*B]."""
    V, B = int(n_views), int(n_bins)
    th = half_turns * math.pi * np.arange(V) / V
    u = (np.arange(B) - (B - 1) / 2.0) * bin_cm
    ct, st = np.cos(th)[:, None], np.sin(th)[:, None]
    out = np.zeros((V, B))
    for cx, cy, a, b, phi, rho in ell:
        r2 = (a * np.cos(th - phi)) ** 2 + (b * np.sin(th - phi)) ** 2
        t = u[None, :] - (cx * ct + cy * st)
        rem = r2[:, None] - t * t
        chord = np.where(rem > 0, 2.0 * a * b * np.sqrt(np.maximum(rem, 0.0)) / r2[:, None], 0.0)
        out += rho * chord
    return out.ravel()


def expected_counts(line_int, mu, I):
    """Mean counts per window, float64 [Wn * n] (window-major)."""
    mu = np.asarray(mu, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64).reshape(-1, mu.size)
    att = np.exp(-np.outer(np.asarray(line_int, dtype=np.float64), mu))  # [n, K]
    return (att @ I.T).T.ravel()


def poisson_counts(mean, seed):
    """Poisson draws as float32 (exact integers)."""
    rng = np.random.default_rng(int(seed))
    y = rng.poisson(np.asarray(mean, dtype=np.float64))
    if y.max(initial=0) >= 2 ** 24:
        raise ValueError("counts exceed the exact float32 integer range")
    return y.astype(np.float32)


# ------------------------------------------------------- known background

def background_ellipses(radius_cm=FOV_CM / 2):
    """Known materials of a scan (the multi-material setting of the paper's
    appendix, in which all but one material are known): a water-like disc of
    density 1.0 filling 85% of the field and a bone-like ring segment
    (density 1.8) as an off-centre ellipse."""
    R = float(radius_cm)
    return np.array([[0.0, 0.0, 0.85 * R, 0.80 * R, 0.0, 1.0],
                     [0.35 * R, -0.2 * R, 0.12 * R, 0.07 * R, 0.6, 1.8]])


def with_background(P, bg_ell=None):
    """A copy of problem P whose scan also holds known materials: their exact
    line integrals bg (float64 [V*B]) and counts redrawn from the model with
    the total line integral (the unknown material's plus the background's,
    sharing the attenuation curve as in the reparametrised model)."""
    import copy
    ell = background_ellipses() if bg_ell is None else np.asarray(bg_ell, dtype=np.float64)
    bg = analytic_sinogram(ell, P.n_views, P.n_bins, P.bin_cm, P.half_turns)
    Q = copy.copy(P)
    Q.bg = bg
    Q.y = poisson_counts(expected_counts(P.line_int + bg, P.mu, P.I), P.seed_noise + 7)
    return Q


# ------------------------------------------------------------- configurations

def bins_for(n_pix):
    """Detector bins covering the image diagonal: ceil(N sqrt 2)."""
    return int(math.ceil(n_pix * math.sqrt(2.0)))


@dataclass
class Problem:
    """A synthetic single-material polychromatic CT scan."""
    name: str
    n_pix: int
    n_views: int
    n_bins: int
    K: int
    Wn: int
    I0: float
    n_ell: int
    seed_phantom: int
    seed_noise: int
    half_turns: int = 1
    pixel_cm: float = 0.0
    bin_cm: float = 0.0
    mu: np.ndarray = field(default=None, repr=False)
    I: np.ndarray = field(default=None, repr=False)
    ell: np.ndarray = field(default=None, repr=False)
    line_int: np.ndarray = field(default=None, repr=False)
    y: np.ndarray = field(default=None, repr=False)
    x_true: np.ndarray = field(default=None, repr=False)
    bg: np.ndarray = field(default=None, repr=False)     # known materials' line integrals

    @property
    def d(self):
        return self.n_pix * self.n_pix

    @property
    def n(self):
        return self.n_views * self.n_bins


def make_problem(name, n_pix, n_views, n_bins, K, Wn, I0, n_ell, seed_phantom,
                 seed_noise, half_turns=1, pixel_cm=None, with_truth=True, bin_cm=None):
    """Draw the phantom, its analytic sinogram and Poisson counts.  Bins are
    as wide as pixels unless bin_cm says otherwise."""
    pixel_cm = FOV_CM / n_pix if pixel_cm is None else float(pixel_cm)
    bin_cm = pixel_cm if bin_cm is None else float(bin_cm)
    mu, I = spectrum(K, Wn, I0)
    ell = ellipses(n_ell, seed_phantom)
    li = analytic_sinogram(ell, n_views, n_bins, bin_cm, half_turns)
    y = poisson_counts(expected_counts(li, mu, I), seed_noise)
    x_true = phantom_image(ell, n_pix, pixel_cm) if with_truth else None
    return Problem(name, int(n_pix), int(n_views), int(n_bins), int(K), int(Wn),
                   float(I0), int(n_ell), int(seed_phantom), int(seed_noise),
                   int(half_turns), pixel_cm, bin_cm, mu, I, ell, li, y, x_true)


# The three single-problem workloads: sizes, spectra and seeds.
CONFIGS = {
    "small_64": dict(n_pix=64, n_views=60, n_bins=92, K=10, Wn=2, I0=1e4,
                     n_ell=8, seed_phantom=101, seed_noise=102),
    "solve_512": dict(n_pix=512, n_views=180, n_bins=725, K=30, Wn=3, I0=1e4,
                      n_ell=20, seed_phantom=201, seed_noise=202),
    "large_1024": dict(n_pix=1024, n_views=720, n_bins=1448, K=64, Wn=4, I0=1e3,
                       n_ell=40, seed_phantom=301, seed_noise=302),
}


def config_problem(name, **over):
    kw = dict(CONFIGS[name])
    kw.update(over)
    return make_problem(name, **kw)


def batch_draws(count=64, seed=401):
    """Shapes of the uneven batch: N in {128..768}, V in [30,360],
    K in [10,64], Wn in [2,4]; B = ceil(N sqrt 2)."""
    rng = np.random.default_rng(int(seed))
    Ns = rng.choice([128, 256, 384, 512, 768], size=count)
    Vs = rng.integers(30, 361, size=count)
    Ks = rng.integers(10, 65, size=count)
    Ws = rng.integers(2, 5, size=count)
    return [dict(n_pix=int(Ns[p]), n_views=int(Vs[p]), n_bins=bins_for(int(Ns[p])),
                 K=int(Ks[p]), Wn=int(Ws[p]), I0=1e4, n_ell=20,
                 seed_phantom=1000 + p, seed_noise=2000 + p)
            for p in range(count)]


def served_stream(count=300, rate=20.0, seed=501):
    """Request parameters of the served stream: Poisson arrivals at `rate`
    per second; per request, independent uniform draws of N in
    {256, 512, 1024}, V in {90, 180, 360}, I0 in {1e3, 1e4} and tolerance in
    {1e-3, 1e-4}; K = 30, Wn = 3, 20 ellipses, seeds 3000+q / 4000+q."""
    rng = np.random.default_rng(int(seed))
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ns = rng.choice([256, 512, 1024], size=count)
    Vs = rng.choice([90, 180, 360], size=count)
    I0s = rng.choice([1e3, 1e4], size=count)
    tols = rng.choice([1e-3, 1e-4], size=count)
    return [dict(arrival=float(arrivals[q]), tol=float(tols[q]),
                 params=dict(n_pix=int(Ns[q]), n_views=int(Vs[q]), n_bins=bins_for(int(Ns[q])),
                             K=30, Wn=3, I0=float(I0s[q]), n_ell=20, seed_phantom=3000 + q,
                             seed_noise=4000 + q))
            for q in range(count)]
