"""The request loop on the GPU: requests arriving while others run are
admitted as memory (and, with the shortest-expected-work policy, the cap on
work in flight) allows; every result equals the same scan solved alone
(bitwise; same step size, formed by the library from the cached lambda_max)
and the CPU oracle's EXACT run of the same step count (paper Sec. 1.2, eq.
extragrad-method) at 1e-4 relative L2."""
import numpy as np
import pytest

from paper_2503_19925_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


SHAPES = [(64, 40, 92, 1e-3), (48, 60, 69, 2e-3), (96, 30, 137, 1e-3), (64, 40, 92, 5e-3),
          (80, 25, 114, 2e-3), (48, 60, 69, 1e-3), (32, 90, 46, 2e-3)]


def requests():
    from paper_2503_19925_amd.serve import Request
    reqs = []
    for q, (N, V, B, tol) in enumerate(SHAPES):
        P = synth.make_problem("req%d" % q, N, V, B, 30, 3, 1e4, 6, 3000 + q, 4000 + q,
                               with_truth=False)
        reqs.append(Request(q, 0.002 * q, P, tol=tol, max_iters=3000))
    return reqs


@pytest.mark.parametrize("policy", ["fcfs", "sjf"])
def test_served_results_equal_solo_and_oracle(ora, policy):
    from paper_2503_19925_amd import exact
    from paper_2503_19925_amd.serve import GpuBackend, Server, step_cost, summarize
    exact.load()
    reqs = requests()
    say("served stream", policy, [(r.problem.n_pix, r.problem.n_views, r.tol) for r in reqs])
    be = GpuBackend(1 << 40, capacity=8)
    fps = [be.footprint(r.problem) for r in reqs]
    if policy == "fcfs":
        # room for three of the largest scans at a time: later ones must queue
        budget, cap = 3 * max(fps), None
    else:
        # memory for all; work in flight for about two scans
        budget, cap = sum(fps), 2.0 * max(step_cost(r.problem) for r in reqs)
    srv = Server(be, budget, chunk_steps=8, policy=policy, work_cap=cap)
    res = srv.run(reqs)
    be.close()
    if policy == "fcfs":
        most = 0                                 # most scans that fit together
        while most < len(fps) and sum(sorted(fps)[:most + 1]) <= budget:
            most += 1
        assert 3 <= srv.peak_running <= most < len(reqs)
    else:
        assert srv.peak_load <= cap and srv.peak_running < len(reqs)
    assert any(r.queued > 0 for r in res)
    s = summarize(res)
    print("  summary", s, flush=True)
    for r, q in zip(res, reqs):
        P = q.problem
        g = exact.Geometry(P.n_pix, P.n_views, P.n_bins)
        x = torch.zeros(g.d, device="cuda")
        info = exact.exact_solve(g, P.mu, P.I, torch.as_tensor(P.y, device="cuda"), x,
                                 gamma=r.gamma, max_iters=q.max_iters, tol=q.tol)
        g.close()
        assert r.status == 1 and info["converged"]
        assert info["iters"] == r.iters, (q.rid, info["iters"], r.iters)
        assert np.array_equal(x.cpu().numpy(), r.x), q.rid
        go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
        x_ora, t, _ = ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(P.d), r.gamma,
                             r.iters)
        rel = np.linalg.norm(r.x.astype(np.float64) - x_ora) / np.linalg.norm(x_ora)
        print("  request %d: %d steps, rel L2 vs oracle %.3e" % (q.rid, r.iters, rel), flush=True)
        assert t == r.iters and rel <= 1e-4


def test_library_gamma_is_theorem2(ora):
    """The step size the library forms from a given lambda_max is Theorem 2's
    c / (lambda sum_k J_k mu_k), J_k the window-summed intensities (paper
    Sec. 2.1), the same as the oracle's rule."""
    from paper_2503_19925_amd import exact
    exact.load()
    P = requests()[2].problem
    g = exact.Geometry(P.n_pix, P.n_views, P.n_bins)
    lam, gamma = exact.exact_step_size(g, P.mu, P.I, 100)
    x = torch.zeros(g.d, device="cuda")
    info = exact.exact_solve(g, P.mu, P.I, torch.as_tensor(P.y, device="cuda"), x,
                             lambda_hat=lam, max_iters=1)
    g.close()
    assert info["lambda_hat"] == lam and info["gamma"] == gamma
    assert abs(gamma - ora.step_size(lam, P.mu, P.I)) <= 1e-14 * gamma
