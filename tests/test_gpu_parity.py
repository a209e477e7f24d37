"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (float32 path vs float64 oracle):
  * forward, per ray:  |s - s_ora| <= 1e-5 * (A|x|)_i   (= 1e-5 s_ora for x >= 0)
  * back-projection, per pixel: |g - g_ora| <= 1e-5 * (A^T |r|)_p
  * operator, per pixel: |F - F_ora| <= 1e-5 * (1/n) (A^T (Y + m))_p, m the
    model counts, since r = Y - m is a difference of two large terms
  * iterates after T steps: ||x - x_ora|| / ||x_ora|| <= 1e-4.
The per-element bounds carry an absolute floor of 1e-9 of the largest
element's scale: a ray that passes exactly one pixel outside the image (or a
pixel that such a ray grazes) has true weight 0, which both sides compute in
double as a rounding-level tent value (~1e-14) with no relative accuracy.
Each case prints its name and shape before touching the GPU.
"""
import math
import os

import numpy as np
import pytest

from paper_2503_19925_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print("[case]", *a, flush=True)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float32).ravel()),
                           device=DEV)


def np64(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64).ravel()


def within(got, want, scale, rel=1e-5):
    """|got - want| <= rel * scale + 1e-9 * max(scale), element by element."""
    scale = np.asarray(scale, dtype=np.float64)
    tol = rel * scale + 1e-9 * float(scale.max(initial=0.0)) + 1e-30
    err = np.abs(np.asarray(got, dtype=np.float64) - want)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, "%d elements out of tolerance; worst %s: got %r want %r scale %r" % (
        bad.size, bad[np.argmax((err / tol)[bad])], got[bad[0]], want[bad[0]], scale[bad[0]])


@pytest.fixture(scope="module")
def ex():
    from paper_2503_19925_amd import exact
    exact.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return exact


# (name, N, V, B, bin/pixel ratio, half_turns)
SMALL_SHAPES = [
    ("small_64", 64, 60, 92, 1.0, 1),
    ("ragged", 77, 33, 109, 1.0, 1),
    ("full_turn", 48, 50, 70, 1.0, 2),
    ("wide_bins", 40, 36, 45, 1.3, 1),
    ("narrow_bins", 40, 36, 81, 0.7, 1),
    ("mostly_missed", 16, 8, 200, 1.0, 1),
    ("one_pixel", 1, 3, 3, 1.0, 1),
    ("two_pixels", 2, 5, 4, 1.0, 1),
    ("one_view", 33, 1, 47, 1.0, 1),
    # detectors narrower than the image: the gather's clamped pair rule
    ("narrow_detector", 48, 30, 40, 1.0, 1),
    ("narrow_detector_wide_bins", 31, 7, 11, 2.0, 1),
    # wider images: several blocks of 128 rays per view, the last one ragged.
    # The forward's lanes take two adjacent rays and read their taps by one
    # of three rules, by the view's |P| (bins per pixel along the line):
    # below 1 (narrow bins), 1 to 2, and 2 or more (the 2.0 and 1.6 ratios;
    # at 1.6 the views near 45 degrees pass 2 while the others stay below)
    ("wide_ragged", 130, 33, 184, 1.0, 1),
    ("wide_full_turn", 160, 50, 227, 1.0, 2),
    ("wide_bins_130", 128, 29, 140, 1.3, 1),
    ("narrow_bins_130", 128, 29, 260, 0.7, 1),
    ("mixed_rules_bins", 96, 40, 80, 1.6, 1),
    # detectors far wider than the image, so that most lanes' crossings are
    # clamped into the padding on one side or the other, under each rule:
    # |P| in [1.5, 2.1] (two-tap and separate loads), [0.5, 0.71] (|P| < 1)
    ("mostly_missed_wide_bins", 24, 9, 180, 1.5, 1),
    ("mostly_missed_narrow_bins", 20, 7, 300, 0.5, 1),
]


def geoms(ex, ora, N, V, B, ratio, turns):
    pc = 10.0 / N
    return (ex.Geometry(N, V, B, pixel_cm=pc, bin_cm=pc * ratio, half_turns=turns),
            ora.Geom(N, V, B, pixel_cm=pc, bin_cm=pc * ratio, half_turns=turns))


@pytest.mark.parametrize("case", SMALL_SHAPES, ids=[c[0] for c in SMALL_SHAPES])
def test_forward_backward_per_element(ex, ora, case):
    name, N, V, B, ratio, turns = case
    say("forward/back", name, N, V, B, ratio, turns)
    g, go = geoms(ex, ora, N, V, B, ratio, turns)
    rng = np.random.default_rng(20)
    x = rng.uniform(0, 2, g.d).astype(np.float32)
    s = torch.empty(g.n, device=DEV)
    ex.exact_forward(g, t32(x), s)
    s_ora = ora.forward(go, x)
    scale = ora.forward(go, np.abs(x))
    within(np64(s), s_ora, scale)
    # signed image: scale by A|x|
    xs = rng.normal(size=g.d).astype(np.float32)
    ex.exact_forward(g, t32(xs), s)
    within(np64(s), ora.forward(go, xs), ora.forward(go, np.abs(xs)))
    # back-projection of a signed sinogram
    r = rng.normal(size=g.n).astype(np.float32)
    img = torch.empty(g.d, device=DEV)
    ex.exact_backproject(g, t32(r), img)
    within(np64(img), ora.back(go, r), ora.back(go, np.abs(r)))
    g.close()


@pytest.mark.parametrize("name", ["solve_512", "large_1024"])
def test_projectors_sampled_full_size(ex, ora, name):
    """Full workload sizes, the launch shapes the benchmark times: sampled rays
    and pixels computed one by one by the oracle."""
    P = synth.config_problem(name, with_truth=True)
    say("sampled projectors", name, P.n_pix, P.n_views, P.n_bins)
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    rng = np.random.default_rng(21)
    x = P.x_true.astype(np.float32)
    s = torch.empty(g.n, device=DEV)
    ex.exact_forward(g, t32(x), s)
    rays = np.unique(np.concatenate([rng.integers(0, g.n, 3000),
                                     np.arange(0, P.n_bins), g.n - 1 - np.arange(P.n_bins)]))
    s_ora = ora.forward_rays(go, x, rays)
    within(np64(s)[rays], s_ora, s_ora)
    r = rng.normal(size=g.n).astype(np.float32)
    img = torch.empty(g.d, device=DEV)
    ex.exact_backproject(g, t32(r), img)
    pix = np.unique(np.concatenate([rng.integers(0, g.d, 48), [0, P.n_pix - 1, g.d - 1,
                                                               g.d // 2 + P.n_pix // 2],
                                    whole_tiles(P.n_pix), near_integer_bins(P, 300, rng)]))
    say("  back-projection: %d pixels (5 whole 16x16 tiles, pixels on bin boundaries)"
        % pix.size)
    g_ora = ora.back_pixels(go, r, pix)
    scale = ora.back_pixels(go, np.abs(r), pix)
    within(np64(img)[pix], g_ora, scale)
    g.close()


def whole_tiles(N, T=16):
    """Every pixel of the back-projector's 16 x 16 tiles at the four corners
    and the centre of the image (the corner tiles hold the image's last row
    and column)."""
    c = (N // 2) // T * T
    out = []
    for ty, tx in [(0, 0), (0, N - T), (N - T, 0), (N - T, N - T), (c, c)]:
        iy, ix = np.meshgrid(np.arange(ty, ty + T), np.arange(tx, tx + T), indexing="ij")
        out.append((iy * N + ix).ravel())
    return np.concatenate(out)


def near_integer_bins(P, count, rng):
    """Pixels whose centre projects to within 1e-3 bin of a bin centre for
    some view (the bin pair's boundary: the tent weights there are 1 and 0,
    and the gather picks the pair by truncating t), `count` of them drawn
    with rng.  Geometry as in the header: pixel centres ((ix - c) d,
    (iy - c) d), c = (N - 1)/2; view v at pi v / V; bin coordinate
    t = <centre, (cos, sin)> / bin + (B - 1)/2."""
    N, V, B = P.n_pix, P.n_views, P.n_bins
    c = (N - 1) / 2.0
    xi = (np.arange(N) - c) * P.pixel_cm
    hits = []
    for v in range(0, V, max(1, V // 120)):
        th = np.pi * v / V
        t = (xi[None, :] * np.cos(th) + xi[:, None] * np.sin(th)) / P.bin_cm + (B - 1) / 2.0
        near = np.abs(t - np.round(t)) <= 1e-3
        hits.append(np.flatnonzero(near.ravel()))
    hits = np.unique(np.concatenate(hits))
    return rng.choice(hits, size=min(count, hits.size), replace=False)


@pytest.mark.parametrize("case", [("tiny", 16, 12, 24, 1.0, 1), ("ragged", 21, 7, 31, 1.0, 1),
                                  ("wide_bins", 12, 9, 14, 1.3, 1),
                                  ("narrow_bins", 12, 9, 25, 0.7, 1)], ids=lambda c: c[0])
def test_count_nonzeros(ex, ora, case):
    """exact_count_nonzeros is the number of positive entries of the device's
    A, whose columns are the forward projections of unit images (each entry
    one weight times the view's step, exact); the oracle's A, from
    unquantized crossings, may differ only in entries that are zero up to
    rounding on one side."""
    name, N, V, B, ratio, turns = case
    say("count nonzeros", name, N, V, B, ratio)
    g, go = geoms(ex, ora, N, V, B, ratio, turns)
    cnt = ex.exact_count_nonzeros(g)
    e = torch.zeros(g.d, device=DEV)
    s = torch.empty(g.n, device=DEV)
    A = np.empty((g.n, g.d))
    A_ora = np.empty((g.n, g.d))
    for p in range(g.d):
        e.zero_()
        e[p] = 1.0
        ex.exact_forward(g, e, s)
        A[:, p] = np64(s)
        u = np.zeros(g.d)
        u[p] = 1.0
        A_ora[:, p] = ora.forward(go, u)
    assert cnt == int((A > 0).sum())
    n_ora = int((A_ora > 0).sum())
    tiny = int(((A > 0) & (A < 1e-6 * A.max())).sum() +
               ((A_ora > 0) & (A_ora < 1e-9 * A_ora.max())).sum())
    print("  nnz device %d, oracle %d (its counter %d), rounding-level entries %d"
          % (cnt, n_ora, ora.nnz(go), tiny), flush=True)
    assert abs(cnt - n_ora) <= tiny
    g.close()


def test_projectors_sampled_max_image(ex, ora):
    """The largest image the ABI accepts (16384^2, 1 GiB as float32) with
    three views and a detector covering it: sampled rays (every one walks
    16384 lines) and pixels against the oracle, one by one."""
    N, V, B = 16384, 3, 23172
    say("sampled projectors at the maximum image size", N, V, B)
    g = ex.Geometry(N, V, B)
    go = ora.Geom(N, V, B)
    rng = np.random.default_rng(31)
    x = rng.random(N * N, dtype=np.float32)
    s = torch.empty(g.n, device=DEV)
    ex.exact_forward(g, t32(x), s)
    rays = np.unique(np.concatenate([rng.integers(0, g.n, 60), [0, B // 2, B - 1, g.n - 1,
                                                                g.n - B // 2]]))
    s_ora = ora.forward_rays(go, x, rays)
    within(np64(s)[rays], s_ora, s_ora)
    del s
    r = rng.normal(size=g.n).astype(np.float32)
    img = torch.empty(g.d, device=DEV)
    ex.exact_backproject(g, t32(r), img)
    pix = np.unique(np.concatenate([rng.integers(0, g.d, 40), [0, N - 1, g.d - N, g.d - 1,
                                                               g.d // 2 + N // 2]]))
    g_ora = ora.back_pixels(go, r, pix)
    within(np64(img)[pix], g_ora, ora.back_pixels(go, np.abs(r), pix))
    del img
    g.close()
    torch.cuda.empty_cache()


def test_adjoint_identity_on_gpu(ex):
    """<A x, y> = <x, A^T y> with the GPU's own projector pair: the weights are
    identical, so only float32 summation order separates the two."""
    N, V, B = 256, 90, 363
    say("adjoint", N, V, B)
    g = ex.Geometry(N, V, B)
    rng = np.random.default_rng(22)
    x = rng.uniform(0, 1, g.d).astype(np.float32)
    y = rng.uniform(0, 1, g.n).astype(np.float32)
    s = torch.empty(g.n, device=DEV)
    img = torch.empty(g.d, device=DEV)
    ex.exact_forward(g, t32(x), s)
    ex.exact_backproject(g, t32(y), img)
    lhs = np.dot(np64(s), y.astype(np.float64))
    rhs = np.dot(x.astype(np.float64), np64(img))
    assert abs(lhs - rhs) <= 2e-7 * abs(lhs)
    g.close()


@pytest.mark.parametrize("case", [
    ("bins_as_wide_as_pixels", 20, 7, 29, 1.0),     # forward: one 16-byte load per lane
    ("narrow_bins", 20, 7, 60, 0.45),               # |P| < 1; gather over a reach of bins
    ("wide_bins", 20, 7, 12, 2.5),                  # |P| >= 2: one 8-byte load per ray
], ids=lambda c: c[0])
def test_forward_matrix_equals_gather_matrix(ex, case):
    """Every entry of A, read column by column from the forward projector
    (one-hot images) and row by row from the gather back-projector (one-hot
    sinograms), is the same float: both sides form the tent weight 1 - |f - j|
    exactly and round it once, then multiply by the same float path length,
    and a one-hot input leaves one nonzero term in every sum."""
    name, N, V, B, ratio = case
    say("matrix", name, N, V, B)
    g = ex.Geometry(N, V, B, pixel_cm=0.1, bin_cm=0.1 * ratio)
    Af = np.zeros((g.n, g.d), dtype=np.float32)
    Ab = np.zeros((g.n, g.d), dtype=np.float32)
    x = torch.zeros(g.d, device=DEV)
    s = torch.empty(g.n, device=DEV)
    for j in range(g.d):
        x.zero_()
        x[j] = 1.0
        ex.exact_forward(g, x, s)
        Af[:, j] = s.cpu().numpy()
    r = torch.zeros(g.n, device=DEV)
    img = torch.empty(g.d, device=DEV)
    for i in range(g.n):
        r.zero_()
        r[i] = 1.0
        ex.exact_backproject(g, r, img)
        Ab[i, :] = img.cpu().numpy()
    torch.cuda.synchronize()
    g.close()
    assert np.count_nonzero(Af) > 2 * g.n
    diff = np.nonzero(Af.view(np.uint32) != Ab.view(np.uint32))
    assert diff[0].size == 0, "%d entries differ; first (ray, pixel) %s: %r vs %r" % (
        diff[0].size, (diff[0][0], diff[1][0]), Af[diff][0], Ab[diff][0])


def test_determinism(ex):
    N, V, B = 128, 45, 182
    say("determinism", N, V, B)
    g = ex.Geometry(N, V, B)
    rng = np.random.default_rng(23)
    x = t32(rng.uniform(0, 1, g.d))
    r = t32(rng.normal(size=g.n))
    s1, s2 = torch.empty(g.n, device=DEV), torch.empty(g.n, device=DEV)
    i1, i2 = torch.empty(g.d, device=DEV), torch.empty(g.d, device=DEV)
    ex.exact_forward(g, x, s1)
    ex.exact_forward(g, x, s2)
    ex.exact_backproject(g, r, i1)
    ex.exact_backproject(g, r, i2)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2) and torch.equal(i1, i2)
    g.close()


def _problem(ex, ora, name, **over):
    P = synth.config_problem(name, **over)
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins, pixel_cm=P.pixel_cm, bin_cm=P.bin_cm)
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins, pixel_cm=P.pixel_cm, bin_cm=P.bin_cm)
    return P, g, go


# (config, overrides): the large workload's spectrum and dose (K = 64, Wn = 4,
# I0 = 1e3) at a reduced size, so every pixel can be checked
OPERATOR_CASES = {"small_64": ("small_64", {}), "solve_512": ("solve_512", {}),
                  "lowdose_256": ("large_1024", dict(n_pix=256, n_views=180, n_bins=363,
                                                     n_ell=20))}


@pytest.mark.parametrize("name", sorted(OPERATOR_CASES))
def test_operator_parity(ex, ora, name):
    cfg, over = OPERATOR_CASES[name]
    P, g, go = _problem(ex, ora, cfg, **over)
    say("operator", name, P.n_pix, P.n_views, P.n_bins, P.K, P.Wn)
    y64 = P.y.astype(np.float64)
    x = (0.9 * P.x_true).astype(np.float32)
    F = torch.empty(g.d, device=DEV)
    r = torch.empty(g.n, device=DEV)
    ex.exact_operator(g, P.mu, P.I, t32(P.y), t32(x), F, r)
    F_ora, s_ora, r_ora = ora.operator(go, P.mu, P.I, y64, x, want_sr=True)
    _, m = ora.residual(s_ora, P.mu, P.I, y64)
    Y = y64.reshape(P.Wn, -1).sum(0)
    scale = ora.back(go, Y + m) / g.n
    within(np64(F), F_ora, scale)
    within(np64(r), r_ora, Y + m)
    g.close()


def test_operator_with_known_background(ex, ora):
    """Known materials (the appendix's reparametrised model): the GPU adds
    bg_i inside every exponential; the oracle builds each ray's
    reparametrised window spectrum."""
    P = synth.with_background(synth.config_problem("small_64"))
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    say("operator with background", P.n_pix, P.n_views, P.n_bins)
    y64 = P.y.astype(np.float64)
    bg32 = P.bg.astype(np.float32)
    x = (0.9 * P.x_true).astype(np.float32)
    F = torch.empty(g.d, device=DEV)
    r = torch.empty(g.n, device=DEV)
    ex.exact_operator(g, P.mu, P.I, t32(P.y), t32(x), F, r, background=t32(bg32))
    F_ora, s_ora, r_ora = ora.operator(go, P.mu, P.I, y64, x, want_sr=True, bg=bg32)
    _, m = ora.residual(s_ora, P.mu, P.I, y64, bg=bg32)
    Y = y64.reshape(P.Wn, -1).sum(0)
    within(np64(F), F_ora, ora.back(go, Y + m) / g.n)
    within(np64(r), r_ora, Y + m)
    g.close()


def test_solve_with_known_background(ex, ora):
    P = synth.with_background(synth.config_problem("small_64"))
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    say("solve with background", P.n_pix, "T = 100")
    gamma = oracle_gamma(ora, go, P)
    bg32 = P.bg.astype(np.float32)
    x = torch.zeros(g.d, device=DEV)
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=gamma, max_iters=100,
                          background=t32(bg32))
    assert info["iters"] == 100
    x_ora, _, _ = ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(g.d), gamma, 100,
                         bg=bg32)
    rel = np.linalg.norm(np64(x) - x_ora) / np.linalg.norm(x_ora)
    print("  rel L2 vs oracle with background after 100 steps: %.3e" % rel, flush=True)
    assert rel <= 1e-4
    bad = bg32.copy()
    bad[5] = -1.0
    with pytest.raises(ex.ExactError):
        ex.exact_solve(g, P.mu, P.I, t32(P.y), torch.zeros(g.d, device=DEV), gamma=gamma,
                       max_iters=2, background=t32(bad))
    g.close()


def test_operator_at_zero_and_monotone(ex, ora):
    """F(0) = (1/n) A^T (Y - I0) (h(0) = 1) and <F(x)-F(z), x-z> >= 0 on the GPU."""
    P, g, go = _problem(ex, ora, "small_64")
    say("operator closed form + monotone", P.n_pix)
    F0 = torch.empty(g.d, device=DEV)
    ex.exact_operator(g, P.mu, P.I, t32(P.y), torch.zeros(g.d, device=DEV), F0)
    Y = P.y.astype(np.float64).reshape(P.Wn, -1).sum(0)
    expect = ora.back(go, Y - P.I0) / g.n
    scale = ora.back(go, Y + P.I0) / g.n
    within(np64(F0), expect, scale)
    rng = np.random.default_rng(24)
    Fx, Fz = torch.empty(g.d, device=DEV), torch.empty(g.d, device=DEV)
    for _ in range(3):
        x = np.maximum(0, P.x_true + rng.normal(scale=0.2, size=g.d)).astype(np.float32)
        z = rng.uniform(0, 1.5, g.d).astype(np.float32)
        ex.exact_operator(g, P.mu, P.I, t32(P.y), t32(x), Fx)
        ex.exact_operator(g, P.mu, P.I, t32(P.y), t32(z), Fz)
        assert np.dot(np64(Fx) - np64(Fz), x.astype(np.float64) - z) >= 0
    g.close()


def test_step_size_matches_oracle(ex, ora):
    P, g, go = _problem(ex, ora, "small_64")
    say("power iteration", P.n_pix)
    lam, gamma = ex.exact_step_size(g, P.mu, P.I, max_iters=300)
    lam_ora, _ = ora.power(go, 3000, 1e-11)
    assert abs(lam - lam_ora) <= 1e-4 * lam_ora
    assert abs(gamma - ora.step_size(lam, P.mu, P.I)) <= 1e-12 * gamma
    g.close()


def oracle_gamma(ora, go, P, power=True):
    """Step size from the oracle: Theorem 2's gamma with lambda_max from power
    iteration, or (cheap, for full-size problems) with the upper bound
    lambda_max(A^T A) <= max row sum * max column sum of A."""
    if power:
        lam, _ = ora.power(go, 1000, 1e-9)
    else:
        rows = ora.forward(go, np.ones(go.d))
        cols = ora.back(go, np.ones(go.n))
        lam = rows.max() * cols.max() / go.n
    return ora.step_size(lam, P.mu, P.I)


def _solve_case(ex, ora, name, T, power=True, **over):
    P, g, go = _problem(ex, ora, name, **over)
    say("solve", name, P.n_pix, P.n_views, P.n_bins, "T =", T)
    gamma = oracle_gamma(ora, go, P, power)
    x = torch.zeros(g.d, device=DEV)
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=gamma, max_iters=T)
    assert info["iters"] == T
    x_ora, t, _ = ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(g.d), gamma, T)
    rel = np.linalg.norm(np64(x) - x_ora) / np.linalg.norm(x_ora)
    print("  rel L2 vs oracle after %d steps: %.3e" % (T, rel), flush=True)
    g.close()
    return rel


def test_solve_parity_small_64(ex, ora):
    assert _solve_case(ex, ora, "small_64", 100) <= 1e-4


def test_solve_parity_mid_128(ex, ora):
    rel = _solve_case(ex, ora, "small_64", 200, power=False, n_pix=128, n_views=90, n_bins=182,
                      K=30, Wn=3)
    assert rel <= 1e-4


def test_solve_parity_lowdose_256(ex, ora):
    """The large workload's spectrum and dose (K = 64 energy bins, 4 windows,
    I0 = 1e3) at 256^2 x 180 views: 50 steps."""
    rel = _solve_case(ex, ora, "large_1024", 50, power=False, n_pix=256, n_views=180,
                      n_bins=363, n_ell=20)
    assert rel <= 1e-4


def _golden(name):
    """Header values and [section] rows of a stored oracle run."""
    head, sec, cur = {}, {}, None
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            sec[cur] = []
        elif "=" in line and cur is None:
            k, v = line.split("=")
            head[k.strip()] = float(v)
        else:
            sec[cur].append([float(t) for t in line.split()])
    return head, {k: np.array(v) for k, v in sec.items()}


def test_large_1024_against_stored_oracle_run(ex):
    """The large low-dose workload at full size (1024^2, 720 views, 1448
    bins, K = 64, Wn = 4, I0 = 1e3) against the oracle's values stored in
    tests/golden/large_1024.txt (written by make_large_1024.py from the
    oracle alone): the operator and the residual at x = float32(0.9 x_true)
    per element at the parity bar on 4096 sampled pixels and rays, and three
    EG steps from x = 0 (the step size stored with them) at 1e-4 relative
    L2 over the sampled pixels."""
    head, sec = _golden("large_1024.txt")
    P = synth.config_problem("large_1024", with_truth=True)
    assert float(P.y.astype(np.float64).sum()) == head["y_sum"]
    say("large_1024 vs stored oracle run", P.n_pix, P.n_views, P.n_bins)
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    F = torch.empty(g.d, device=DEV)
    r = torch.empty(g.n, device=DEV)
    ex.exact_operator(g, P.mu, P.I, t32(P.y), t32((0.9 * P.x_true).astype(np.float32)), F, r)
    fp = sec["F"]
    within(np64(F)[fp[:, 0].astype(np.int64)], fp[:, 1], fp[:, 2])
    rr = sec["r"]
    within(np64(r)[rr[:, 0].astype(np.int64)], rr[:, 1], rr[:, 2])
    x = torch.zeros(g.d, device=DEV)
    steps = int(head["steps"])
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=head["gamma"], max_iters=steps)
    assert info["iters"] == steps
    xs = np64(x)
    xp = sec["x"]
    pix, val = xp[:, 0].astype(np.int64), xp[:, 1]
    rel = np.linalg.norm(xs[pix] - val) / np.linalg.norm(val)
    nrm = abs(np.linalg.norm(xs) - head["x_norm"]) / head["x_norm"]
    print("  %d steps: sampled rel L2 %.3e, norm rel %.3e (oracle float build drift %.3e)"
          % (steps, rel, nrm, head["f32_rel_l2"]), flush=True)
    assert rel <= 1e-4 and nrm <= 1e-4
    g.close()


def test_solve_parity_narrow_detector(ex, ora):
    """A detector narrower than the image: the update kernels take the
    clamped pair rule."""
    rel = _solve_case(ex, ora, "small_64", 60, n_pix=48, n_views=30, n_bins=40)
    assert rel <= 1e-4


def test_solve_parity_narrow_bins(ex, ora):
    """Bins 0.7 pixels wide: the update kernels take the general rule (every
    bin within reach of the nearest)."""
    rel = _solve_case(ex, ora, "small_64", 60, n_pix=40, n_views=36, n_bins=81,
                      bin_cm=0.7 * 10.0 / 40)
    assert rel <= 1e-4


def test_solve_parity_full_512_two_steps(ex, ora):
    """The benchmark's workload at full size, two full steps (8 projector
    passes on the oracle)."""
    assert _solve_case(ex, ora, "solve_512", 2, power=False) <= 1e-5


def test_solve_stop_rule(ex, ora):
    P, g, go = _problem(ex, ora, "small_64")
    say("solve stop rule", P.n_pix)
    gamma = oracle_gamma(ora, go, P)
    tol = 2e-3
    x_ora, t_ora, hist = ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(g.d), gamma,
                                5000, tol=tol)
    x = torch.zeros(g.d, device=DEV)
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=gamma, max_iters=5000, tol=tol,
                          check_every=7)
    assert info["converged"]
    assert info["resid"] <= tol
    assert abs(info["iters"] - t_ora) <= 1, (info["iters"], t_ora)
    # the iterate against the oracle's run of exactly the GPU's step count
    # (the same as x_ora when the stop steps coincide)
    x_at, _, _ = ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(g.d), gamma,
                        info["iters"])
    assert np.linalg.norm(np64(x) - x_at) <= 1e-4 * np.linalg.norm(x_at)
    # a cap below the stopping step reports non-convergence
    x2 = torch.zeros(g.d, device=DEV)
    info2 = ex.exact_solve(g, P.mu, P.I, t32(P.y), x2, gamma=gamma, max_iters=5, tol=tol)
    assert info2["converged"] is False and info2["iters"] == 5
    g.close()


@pytest.fixture(scope="module")
def small_gamma(ora):
    P = synth.config_problem("small_64")
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    return oracle_gamma(ora, go, P)


@pytest.mark.parametrize("T,start", [(0, "half"), (1, "zero"), (2, "half"), (9, "zero"),
                                     (100, "zero"), (101, "half")])
def test_solve_averaged_iterate_parity(ex, ora, small_gamma, T, start):
    """The averaged iterate (mean of x_j, j = floor(s/2)+1 .. s) after T fixed
    steps, against the oracle's direct mean of its stored trajectory.  At
    T = 100 the device keeps 27 ring slots for the 50 iterates a window ever
    drops, so the ring wraps."""
    P, g, go = _problem(ex, ora, "small_64")
    say("averaged iterate", P.n_pix, "T =", T, "start", start)
    x1 = np.zeros(g.d) if start == "zero" else (0.5 * P.x_true).astype(np.float32).astype(np.float64)
    x = t32(x1)
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=small_gamma, max_iters=T,
                          stop_mode=ex.STOP_AVERAGED_ITERATE, check_every=8)
    xb_ora, t, crit, _ = ora.eg_avg(go, P.mu, P.I, P.y.astype(np.float64), x1, small_gamma, T)
    assert info["iters"] == T == t
    got = np64(x)
    if T == 0:
        np.testing.assert_array_equal(got, x1)
    else:
        rel = np.linalg.norm(got - xb_ora) / np.linalg.norm(xb_ora)
        print("  averaged iterate rel L2 %.3e; criterion %.6e vs %.6e" % (
            rel, info["resid"], crit[-1]), flush=True)
        assert rel <= 1e-4
        assert abs(info["resid"] - crit[-1]) <= 1e-3 * crit[-1]
    g.close()


def test_solve_averaged_stop_rule(ex, ora, small_gamma):
    """The averaged rule stops at the first step with ||xbar_{t+1} - xbar_t||
    <= tol (absolute).  The criterion alternates between window moves that
    only add an iterate and moves that also drop one, so a marginal float
    difference can move the stop by two steps."""
    P, g, go = _problem(ex, ora, "small_64")
    say("averaged stop rule", P.n_pix)
    tol = 0.02
    xb_ora, t_ora, crit, _ = ora.eg_avg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(g.d),
                                        small_gamma, 1000, tol=tol)
    assert t_ora < 1000
    x = torch.zeros(g.d, device=DEV)
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=small_gamma, max_iters=1000, tol=tol,
                          stop_mode=ex.STOP_AVERAGED_ITERATE, check_every=5)
    assert info["converged"] and info["resid"] <= tol
    assert abs(info["iters"] - t_ora) <= 2, (info["iters"], t_ora)
    # the averaged iterate against the oracle's of exactly the GPU's step count
    xb_at, t_at, _, _ = ora.eg_avg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(g.d),
                                   small_gamma, info["iters"])
    assert t_at == info["iters"]
    assert np.linalg.norm(np64(x) - xb_at) <= 1e-4 * np.linalg.norm(xb_at)
    g.close()


def test_solve_is_deterministic(ex):
    P = synth.config_problem("small_64")
    say("solve determinism")
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    x1, x2 = torch.zeros(g.d, device=DEV), torch.zeros(g.d, device=DEV)
    i1 = ex.exact_solve(g, P.mu, P.I, t32(P.y), x1, max_iters=50)
    i2 = ex.exact_solve(g, P.mu, P.I, t32(P.y), x2, max_iters=50)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and i1["gamma"] == i2["gamma"]
    g.close()


def test_solver_profile_steps_equal_graph_steps(ex):
    """exact_solver_profile launches the step's kernels one by one with
    events between them: the iterates equal those of graph replays and the
    five phase times are positive."""
    P = synth.config_problem("small_64")
    say("solver profile vs graph steps")
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    y = t32(P.y)
    xa, xb = torch.zeros(g.d, device=DEV), torch.zeros(g.d, device=DEV)
    sa = ex.Solver(g, P.mu, P.I, y, xa, max_iters=10)
    sa.step(10)
    _, ia = sa.poll()
    sb = ex.Solver(g, P.mu, P.I, y, xb, max_iters=10)
    sb.step(4)
    ms = sb.profile(6)
    _, ib = sb.poll()
    assert ia["iters"] == ib["iters"] == 10
    assert len(ms) == ex.STEP_PHASES and all(t > 0 for t in ms), ms
    assert torch.equal(xa, xb)
    sa.close()
    sb.close()
    g.close()


def test_solver_step_grouping_is_bitwise_neutral(ex):
    """A solver's steps run as replays of an eight-step graph and then of a
    one-step graph for the rest: 13 steps in one call, 5 then 8, and 13 one
    at a time give bitwise the same iterate and state; and a run that stops
    inside an eight-step replay (max_iters 11) stops at its step with the
    iterate of an eleven-step run."""
    P = synth.config_problem("small_64")
    say("solver step grouping")
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    y = t32(P.y)
    xs, infos = [], []
    for calls in ([13], [5, 8], [1] * 13):
        x = torch.zeros(g.d, device=DEV)
        sv = ex.Solver(g, P.mu, P.I, y, x, max_iters=100)
        for n in calls:
            sv.step(n)
        _, info = sv.poll()
        torch.cuda.synchronize()
        xs.append(x)
        infos.append(info)
        sv.close()
    assert all(i["iters"] == 13 for i in infos), infos
    assert all(torch.equal(xs[0], x) for x in xs[1:])
    assert all(i["resid"] == infos[0]["resid"] for i in infos)
    # stopping inside a replay: later steps of the graph are no-ops
    xa, xb = torch.zeros(g.d, device=DEV), torch.zeros(g.d, device=DEV)
    sa = ex.Solver(g, P.mu, P.I, y, xa, max_iters=11)
    sa.step(16)
    _, ia = sa.poll()
    sb = ex.Solver(g, P.mu, P.I, y, xb, max_iters=100)
    for _ in range(11):
        sb.step(1)
    _, ib = sb.poll()
    torch.cuda.synchronize()
    assert ia["iters"] == ib["iters"] == 11
    assert torch.equal(xa, xb)
    sa.close()
    sb.close()
    g.close()


def test_scalar_worked_example_on_gpu(ex):
    """The hand-worked one-pixel example (tests/golden/eg_scalar.txt)."""
    say("scalar EG example")
    golden = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "eg_scalar.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            golden[k.strip()] = float(v)
    g = ex.Geometry(1, 1, 1, pixel_cm=1.0, bin_cm=1.0)
    s = torch.empty(1, device=DEV)
    ex.exact_forward(g, t32([2.5]), s)
    assert np64(s)[0] == 2.5
    x = torch.zeros(1, device=DEV)
    y = t32([math.exp(-1.0)])
    ex.exact_solve(g, [1.0], [1.0], y, x, gamma=0.5, max_iters=1)
    assert abs(np64(x)[0] - golden["x_2"]) <= 2e-7
    ex.exact_solve(g, [1.0], [1.0], y, x, gamma=0.5, max_iters=1)
    assert abs(np64(x)[0] - golden["x_3"]) <= 4e-7
    x0 = torch.zeros(1, device=DEV)
    ex.exact_solve(g, [1.0], [1.0], t32([1.5]), x0, gamma=0.5, max_iters=3)
    assert np64(x0)[0] == 0.0
    g.close()


def test_error_paths(ex):
    say("error paths")
    g = ex.Geometry(16, 10, 23)
    x = torch.zeros(g.d, device=DEV)
    y = torch.ones(2 * g.n, device=DEV)
    F = torch.empty(g.d, device=DEV)
    with pytest.raises(ex.ExactError):
        ex.exact_operator(g, [0.2, -1.0], [1.0, 1.0, 1.0, 1.0], y, x, F)      # mu <= 0
    with pytest.raises(ex.ExactError):
        ex.exact_operator(g, [0.2, 0.3], [0.0, 0.0, 1.0, 1.0], y, x, F)       # empty window
    with pytest.raises(ex.ExactError):
        ex.exact_operator(g, np.ones(200), np.ones(400), torch.ones(2 * g.n, device=DEV), x, F)
    bad = torch.ones(2 * g.n, device=DEV)
    bad[5] = -1.0
    with pytest.raises(ex.ExactError):
        ex.exact_solve(g, [0.2, 0.3], [1.0, 1.0, 1.0, 1.0], bad, x, max_iters=3)
    bad[5] = float("nan")
    with pytest.raises(ex.ExactError):
        ex.exact_solve(g, [0.2, 0.3], [1.0, 1.0, 1.0, 1.0], bad, x, max_iters=3)
    xneg = torch.zeros(g.d, device=DEV)
    xneg[3] = -0.5
    with pytest.raises(ex.ExactError):
        ex.exact_solve(g, [0.2, 0.3], [1.0, 1.0, 1.0, 1.0], y, xneg, max_iters=3)
    assert np64(xneg)[3] == -0.5
    # zero steps leave x unchanged
    x1 = torch.full((g.d,), 0.25, device=DEV)
    info = ex.exact_solve(g, [0.2, 0.3], [1.0, 1.0, 1.0, 1.0], y, x1, gamma=1e-3, max_iters=0)
    assert info["iters"] == 0 and (np64(x1) == 0.25).all()
    g.close()


def test_solve_parity_full_512_500_steps(ex):
    """The benchmark's workload at full size for 500 steps against the oracle's
    run stored in tests/golden/trajectory_solve_512.txt (written by
    make_trajectory_512.py from the oracle alone): relative L2 over 4096
    sampled pixels and the iterate's norm within 1e-4."""
    path = os.path.join(os.path.dirname(__file__), "golden", "trajectory_solve_512.txt")
    head, pix, val = {}, [], []
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if "=" in line:
            k, v = line.split("=")
            head[k.strip()] = float(v)
        else:
            p, v = line.split()
            pix.append(int(p))
            val.append(float(v))
    pix, val = np.array(pix), np.array(val)
    P = synth.config_problem("solve_512", with_truth=False)
    assert float(P.y.astype(np.float64).sum()) == head["y_sum"]
    say("solve 512 x 500 vs stored oracle run")
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    x = torch.zeros(g.d, device=DEV)
    info = ex.exact_solve(g, P.mu, P.I, t32(P.y), x, gamma=head["gamma"], max_iters=int(head["steps"]))
    assert info["iters"] == int(head["steps"])
    xs = np64(x)
    rel = np.linalg.norm(xs[pix] - val) / np.linalg.norm(val)
    nrm = abs(np.linalg.norm(xs) - head["x_norm"]) / head["x_norm"]
    print("  sampled rel L2 %.3e, norm rel %.3e (oracle float build drift %.3e)"
          % (rel, nrm, head["f32_rel_l2"]), flush=True)
    assert rel <= 1e-4 and nrm <= 1e-4
    g.close()
