"""The request loop on the GPU: requests arriving while others run are
admitted as memory frees up, and every result equals the same scan solved
alone (bitwise; same step size)."""
import numpy as np
import pytest

from paper_2503_19925_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def test_served_results_equal_solo():
    from paper_2503_19925_amd import exact
    from paper_2503_19925_amd.serve import GpuBackend, Request, Server, summarize
    exact.load()
    shapes = [(64, 40, 92, 1e-3), (48, 60, 69, 2e-3), (96, 30, 137, 1e-3), (64, 40, 92, 5e-3),
              (80, 25, 114, 2e-3), (48, 60, 69, 1e-3), (32, 90, 46, 2e-3)]
    reqs = []
    for q, (N, V, B, tol) in enumerate(shapes):
        P = synth.make_problem("req%d" % q, N, V, B, 30, 3, 1e4, 6, 3000 + q, 4000 + q,
                               with_truth=False)
        reqs.append(Request(q, 0.002 * q, P, tol=tol, max_iters=3000))
    say("served stream", [(r.problem.n_pix, r.problem.n_views, r.tol) for r in reqs])
    be = GpuBackend(1 << 40, capacity=8)
    # room for three of the largest scans at a time: later ones must queue
    fps = [be.footprint(r.problem) for r in reqs]
    budget = 3 * max(fps)
    srv = Server(be, budget, chunk_steps=8)
    res = srv.run(reqs)
    be.close()
    most = 0                                 # most scans that fit together
    while most < len(fps) and sum(sorted(fps)[:most + 1]) <= budget:
        most += 1
    assert 3 <= srv.peak_running <= most < len(reqs)
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
