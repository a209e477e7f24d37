"""GPU parity of EXACT with an explicit measurement matrix (the Gaussian
measurement model, Sec. 2.2, and its experiment in Sec. 5) against the CPU
oracle, plus the cross-check that the dense operator with the explicit Joseph
matrix is the CT operator.

Tolerances: F per element within 1e-5 of (1/n) |A|^T (Y + m) (the residual is
a difference of two terms of that size); iterates 1e-4 rel L2 after 200
steps; the noiseless Gaussian experiment reaches x* to 1e-4 (float32 data
and the problem's conditioning bound it).
"""
import math

import numpy as np
import pytest

from paper_2503_19925_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print("[case]", *a, flush=True)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float32)), device=DEV)


def np64(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64).ravel()


@pytest.fixture(scope="module")
def ex():
    from paper_2503_19925_amd import exact
    exact.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return exact


def gaussian(d, n, seed, norm=3.0):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, d)).astype(np.float32)
    xs = rng.normal(size=d)
    xs *= norm / np.linalg.norm(xs)
    y = np.exp(-np.maximum(A.astype(np.float64) @ xs, 0.0))
    return A, xs, y


@pytest.mark.parametrize("n,d,K,Wn", [(400, 20, 1, 1), (3000, 300, 7, 2), (2000, 1500, 12, 3),
                                      (1200, 900, 5, 2), (777, 4096, 3, 1), (5, 1, 1, 1)])
def test_dense_operator_parity(ex, ora, n, d, K, Wn):
    say("dense operator", n, d, K, Wn)
    rng = np.random.default_rng(n + d)
    A = rng.normal(size=(n, d)).astype(np.float32)
    mu, I = synth.spectrum(K, Wn, 50.0)
    x = (rng.normal(size=d) * 0.05).astype(np.float32)
    y = rng.poisson(20.0, Wn * n).astype(np.float32)
    F = torch.empty(d, device=DEV)
    ex.exact_dense_operator(t32(A), mu, I, t32(y), t32(x), F)
    A64 = A.astype(np.float64)
    F_ora = ora.dense_operator(A64, mu, I, y.astype(np.float64), x.astype(np.float64))
    s = A64 @ x.astype(np.float64)
    Ik = I.reshape(Wn, K).sum(0)
    m = np.exp(-np.outer(np.maximum(s, 0), mu)) @ Ik
    Y = y.astype(np.float64).reshape(Wn, n).sum(0)
    scale = np.abs(A64).T @ (Y + m) / n
    err = np.abs(np64(F) - F_ora)
    assert (err <= 1e-5 * scale + 1e-9 * scale.max()).all(), err.max()


def test_dense_matches_ct_with_joseph_matrix(ex, ora):
    """The explicit Joseph matrix (pixel by pixel) in the dense path gives the
    CT operator of the matrix-free path."""
    N, V, B = 12, 10, 17
    P = synth.make_problem("dense_ct", N, V, B, 6, 2, 1e4, 4, 5, 6)
    g = ex.Geometry(N, V, B)
    go = ora.Geom(N, V, B)
    say("dense vs CT", N, V, B)
    pc = go.pixel_cm
    c = (N - 1) / 2.0
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    xi, eta = (ix - c) * pc, (iy - c) * pc
    A = np.zeros((V * B, N * N))
    for v in range(V):
        th = math.pi * v / V
        ct, st = math.cos(th), math.sin(th)
        tp = (xi * ct + eta * st).ravel()
        mm = max(abs(ct), abs(st))
        for b in range(B):
            u = (b - (B - 1) / 2.0) * pc
            A[v * B + b] = np.maximum(0.0, 1.0 - np.abs(u - tp) / (pc * mm)) * pc / mm
    x = (0.8 * P.x_true).astype(np.float32)
    Fd = torch.empty(g.d, device=DEV)
    Fc = torch.empty(g.d, device=DEV)
    ex.exact_dense_operator(t32(A), P.mu, P.I, t32(P.y), t32(x), Fd)
    ex.exact_operator(g, P.mu, P.I, t32(P.y), t32(x), Fc)
    Y = P.y.astype(np.float64).reshape(P.Wn, -1).sum(0)
    scale = ora.back(go, Y + Y.max()) / g.n
    assert np.abs(np64(Fd) - np64(Fc)).max() <= 1e-5 * scale.max()
    g.close()


def test_dense_solve_parity(ex, ora):
    A, xs, y = gaussian(20, 400, 11)
    say("dense solve", 400, 20)
    x = torch.zeros(20, device=DEV)
    info = ex.exact_dense_solve(t32(A), [1.0], [1.0], t32(y), x, gamma=0.25, max_iters=200)
    x_ora, t, _ = ora.dense_eg(A.astype(np.float64), [1.0], [1.0], y, np.zeros(20), 0.25, 200)
    assert info["iters"] == t == 200
    rel = np.linalg.norm(np64(x) - x_ora) / np.linalg.norm(x_ora)
    print("  rel L2 after 200 steps %.3e" % rel, flush=True)
    assert rel <= 1e-4
    # a ball smaller than ||x*|| keeps every iterate inside it
    xb = torch.zeros(20, device=DEV)
    ex.exact_dense_solve(t32(A), [1.0], [1.0], t32(y), xb, gamma=0.25, max_iters=200, radius=2.0)
    xb_ora, _, _ = ora.dense_eg(A.astype(np.float64), [1.0], [1.0], y, np.zeros(20), 0.25, 200,
                                radius=2.0)
    assert np.linalg.norm(np64(xb)) <= 2.0 * (1 + 1e-6)
    assert np.linalg.norm(np64(xb) - xb_ora) <= 1e-4 * np.linalg.norm(xb_ora)


def test_dense_gaussian_experiment_converges(ex):
    """The paper's Gaussian experiment (noiseless, monochromatic, ||x*|| = 3,
    gamma = 0.25, n = 40 d): the natural-residual stop fires and the iterate
    is x* to the accuracy that float32 counts (y rounded to 2^-24 relative)
    and the conditioning allow."""
    A, xs, y = gaussian(12, 480, 12)
    say("dense Gaussian experiment", 480, 12)
    x = torch.zeros(12, device=DEV)
    info = ex.exact_dense_solve(t32(A), [1.0], [1.0], t32(y), x, gamma=0.25, max_iters=20000,
                                tol=1e-7)
    err = np.linalg.norm(np64(x) - xs) / 3.0
    print("  %d steps, rel error %.3e" % (info["iters"], err), flush=True)
    assert info["converged"] and info["iters"] < 20000 and err <= 1e-4


def test_dense_power_iteration(ex):
    A, xs, y = gaussian(30, 600, 13)
    say("dense step size", 600, 30)
    x = torch.zeros(30, device=DEV)
    info = ex.exact_dense_solve(t32(A), [1.0], [1.0], t32(y), x, max_iters=1, power_iters=500)
    lam = np.linalg.eigvalsh(A.astype(np.float64).T @ A.astype(np.float64) / 600)[-1]
    assert abs(info["lambda_hat"] - lam) <= 1e-4 * lam
    assert abs(info["gamma"] - 0.25 / lam) <= 1e-4 * info["gamma"]
