"""GPU parity of the TV-ball and orthant projection (the constraint set of the
paper's experiments, Sec. 5) against the CPU oracle.

The projection makes data-dependent decisions (the binary search on the TV
weight compares a TV value with tau; Dykstra's loop compares a step norm with
its tolerance).  Both sides compute those values in double, but from float32
images on the GPU.  The cases here are ones where no decision lies near its
threshold: the tests assert that the GPU took the oracle's decision path
(the same Dykstra rounds and TV-regularized solves) and then compare the
results at 1e-4 relative L2; each result is also checked for the properties
that define it (feasibility, the projection inequality).
"""
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


@pytest.fixture(scope="module")
def ex():
    from paper_2503_19925_amd import exact
    exact.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return exact


def _noisy_phantom(N, seed, noise):
    P = synth.make_problem("tv", N, 8, synth.bins_for(N), 5, 1, 1e4, 6, seed, seed + 1)
    rng = np.random.default_rng(seed + 2)
    z = (P.x_true + rng.normal(scale=noise, size=N * N)).astype(np.float32)
    return P, z


@pytest.mark.parametrize("N", [1, 2, 33, 64, 512])
def test_tv_norm(ex, ora, N):
    say("tv norm", N)
    rng = np.random.default_rng(N)
    x = rng.normal(size=N * N).astype(np.float32)
    got = ex.exact_tv_norm(t32(x))
    want = ora.tv_norm(x.astype(np.float64))
    assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (got, want)


@pytest.mark.parametrize("lam", [0.05, 0.5, 3.0])
def test_tv_prox_parity(ex, ora, lam):
    N = 64
    say("tv prox", N, "lam", lam)
    _, z = _noisy_phantom(N, 71, 0.2)
    x = torch.empty(N * N, device=DEV)
    ex.exact_tv_prox(t32(z), lam, x, iters=100)
    want = ora.tv_prox(z.astype(np.float64), lam, iters=100)
    err = np.abs(np64(x) - want).max()
    print("  max abs err %.3e (|z|max %.3f)" % (err, np.abs(z).max()), flush=True)
    assert err <= 2e-5 * np.abs(z).max()
    # lam = 0 is the identity
    ex.exact_tv_prox(t32(z), 0.0, x)
    assert np.array_equal(np64(x), z.astype(np.float64))


def _check_projection(ora, z, x, tau):
    assert x.min() >= 0
    assert ora.tv_norm(x) <= tau + 0.011
    scale = np.linalg.norm(z - x) * np.linalg.norm(z)
    for w in (0.0 * x, 0.5 * x, 0.9 * x, np.full(x.size, x.mean())):
        assert np.dot(z - x, w - x) <= 2e-3 * scale


@pytest.mark.parametrize("N,frac", [(48, 0.8), (40, 0.5)])
def test_project_tv_parity(ex, ora, N, frac):
    P, z = _noisy_phantom(N, 81 + N, 0.25)
    tau = frac * ora.tv_norm(P.x_true)
    say("project tv", N, "tau", round(tau, 3))
    out = torch.empty(N * N, device=DEV)
    info = ex.exact_project_tv(t32(z), tau, out)
    want, rounds, solves = ora.project_tv(z.astype(np.float64), tau)
    got = np64(out)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("  gpu rounds %d solves %d | oracle rounds %d solves %d | rel L2 %.3e | %.1f ms" % (
        info["rounds"], info["solves"], rounds, solves, rel, info["ms"]), flush=True)
    _check_projection(ora, z.astype(np.float64), got, tau)
    assert (info["rounds"], info["solves"]) == (rounds, solves)
    assert rel <= 1e-4
    assert abs(info["tv"] - ora.tv_norm(got)) <= 1e-9 * info["tv"]


def test_project_tv_feasible_input_unchanged(ex, ora):
    P, _ = _noisy_phantom(32, 91, 0.0)
    x = P.x_true.astype(np.float32)
    tau = ora.tv_norm(x.astype(np.float64)) + 1.0
    say("project tv feasible", 32)
    out = torch.empty(x.size, device=DEV)
    info = ex.exact_project_tv(t32(x), tau, out)
    assert info["rounds"] == 1 and info["solves"] == 0
    assert np.array_equal(np64(out), x.astype(np.float64))


def test_solve_tv_parity(ex, ora):
    """EG over the TV ball and the orthant, three steps at 32^2, against the
    oracle's EG over the same set."""
    P = synth.make_problem("tv_solve", 32, 30, 46, 8, 2, 1e4, 6, 95, 96)
    tau = 0.8 * ora.tv_norm(P.x_true)
    say("solve tv", 32, "tau", round(tau, 3))
    g = ex.Geometry(P.n_pix, P.n_views, P.n_bins)
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    lam, _ = ora.power(go, 1000, 1e-9)
    gamma = ora.step_size(lam, P.mu, P.I)
    # start from a noisy copy of the truth so that the TV constraint is active
    rng = np.random.default_rng(97)
    x1 = np.maximum(0, P.x_true + rng.normal(scale=0.3, size=g.d)).astype(np.float32)
    x = t32(x1)
    info, tinfo = ex.exact_solve_tv(g, P.mu, P.I, t32(P.y), x, tau, gamma=gamma, max_iters=3)
    x_ora, t, _, ns_ora = ora.eg_tv(go, P.mu, P.I, P.y.astype(np.float64),
                                    x1.astype(np.float64), gamma, 3, tau=tau, want_solves=True)
    got = np64(x)
    rel = np.linalg.norm(got - x_ora) / np.linalg.norm(x_ora)
    print("  3 steps: rel L2 %.3e, solves %d (oracle %d), %.1f ms"
          % (rel, tinfo["solves"], ns_ora, info["ms"]), flush=True)
    assert info["iters"] == t == 3
    assert got.min() >= 0 and ora.tv_norm(got) <= tau + 0.011
    assert tinfo["solves"] == ns_ora
    assert rel <= 1e-4
    g.close()
