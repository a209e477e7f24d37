"""Host logic of the request loop (paper_2503_19925_amd.serve) on the CPU,
with a fake backend: admission under an HBM budget (in arrival order, or
shortest expected work first under a cap on work in flight, with aging),
retirement, timing and the summary."""
from types import SimpleNamespace

import pytest

from paper_2503_19925_amd.serve import Request, Server, StepEstimate, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Each request needs problem.need steps; a step costs 1 ms of clock."""

    def __init__(self, clock):
        self.clock = clock
        self.left, self.done_iters, self.order = {}, {}, []
        self.next_slot = 0
        self.max_live = 0

    def footprint(self, P):
        return P.fp

    def add(self, req):
        s = self.next_slot
        self.next_slot += 1
        self.left[s] = req.problem.need
        self.done_iters[s] = 0
        self.order.append(req.rid)
        self.max_live = max(self.max_live, len(self.left))
        return s, 0.5

    def step(self, n):
        self.clock.t += 1e-3 * n
        for s in self.left:
            k = min(n, self.left[s])
            self.left[s] -= k
            self.done_iters[s] += k
        return sum(1 for v in self.left.values() if v > 0)

    def poll(self, slot):
        return (1 if self.left[slot] == 0 else 0), {"iters": self.done_iters[slot], "resid": 1e-5}

    def retire(self, slot):
        del self.left[slot]
        return None


def req(rid, arrival, fp, need, cost=1.0, tol=1e-4):
    P = SimpleNamespace(fp=fp, need=need, cost=cost, n_pix=need, n_views=1, n_bins=1, I0=1.0)
    return Request(rid, arrival, P, tol=tol)


def make(budget, chunk=4, policy="fcfs", **kw):
    clock = FakeClock()
    be = FakeBackend(clock)
    return Server(be, budget, chunk_steps=chunk, realtime=False, clock=clock, policy=policy,
                  cost=lambda P: P.cost, **kw), be


def test_admission_respects_budget_and_order():
    srv, be = make(budget=250)
    reqs = [req(i, 0.0, 100, 10 + i) for i in range(6)]
    res = srv.run(reqs)
    assert [r.rid for r in res] == list(range(6))
    assert be.order == list(range(6))            # admitted in arrival order
    assert be.max_live == 2 and srv.peak_running == 2
    assert all(r.status == 1 for r in res)
    # later requests waited for memory
    assert res[0].queued == 0.0 and res[5].queued > 0.0


def test_no_overtaking_of_a_large_request():
    srv, be = make(budget=300)
    reqs = [req(0, 0.0, 200, 40), req(1, 0.0, 250, 8), req(2, 0.0, 50, 8)]
    srv.run(reqs)
    # request 2 would fit beside 0 but must not overtake 1
    assert be.order == [0, 1, 2]


def test_idle_gaps_and_latency():
    srv, be = make(budget=1000)
    reqs = [req(0, 0.0, 10, 8), req(1, 5.0, 10, 8)]
    res = srv.run(reqs)
    assert res[1].admitted >= 5.0
    assert abs(res[1].latency - 8e-3) < 1e-9     # no queueing, 8 steps of 1 ms
    s = summarize(res)
    assert s["requests"] == 2 and s["p99_s"] >= s["p50_s"] > 0


def test_oversized_request_rejected():
    srv, _ = make(budget=100)
    with pytest.raises(ValueError):
        srv.run([req(0, 0.0, 101, 5)])


def test_summary_percentiles():
    srv, _ = make(budget=10 ** 6, chunk=1)
    res = srv.run([req(i, 0.0, 1, 1 + i) for i in range(100)])
    s = summarize(res)
    assert abs(s["p50_s"] - 0.0505) < 2e-3 and s["p99_s"] <= 0.1 + 1e-9
    assert s["mean_iters"] == pytest.approx(50.5)


def test_sjf_admits_least_expected_work_first():
    """Expected work = expected steps (prior per tolerance) x step cost: the
    cheapest waiting scan goes first, ties in arrival order."""
    srv, be = make(budget=10 ** 6, policy="sjf", work_cap=1.0,
                   estimate=StepEstimate(prior={1e-3: 100, 1e-4: 1000}))
    reqs = [req(0, 0.0, 1, 40, cost=1.0, tol=1e-4),     # 1000
            req(1, 0.0, 1, 40, cost=4.0, tol=1e-3),     # 400
            req(2, 0.0, 1, 40, cost=1.0, tol=1e-3),     # 100
            req(3, 0.0, 1, 40, cost=1.0, tol=1e-3)]     # 100
    srv.run(reqs)
    assert be.order == [2, 3, 1, 0]
    assert be.max_live == 1                       # the cap holds one scan of cost >= 1


def test_sjf_work_cap_and_first_admission():
    """Scans are admitted while their summed step cost stays within the cap;
    a scan costlier than the cap still runs when nothing else does."""
    srv, be = make(budget=10 ** 6, policy="sjf", work_cap=3.0)
    reqs = [req(i, 0.0, 1, 20, cost=1.0) for i in range(5)] + [req(5, 0.0, 1, 20, cost=7.0)]
    res = srv.run(reqs)
    assert be.max_live == 3 and srv.peak_load <= 7.0
    assert all(r.status == 1 for r in res)
    assert be.order[-1] == 5


def test_sjf_learns_step_counts_per_class():
    """After a scan of a class finishes, its measured steps replace the prior."""
    est = StepEstimate(default=1000.0)
    srv, be = make(budget=10 ** 6, policy="sjf", work_cap=1.0, estimate=est)
    a = req(0, 0.0, 1, 8, cost=1.0)
    srv.run([a])
    assert est.expect(a) == 8
    b = req(1, 0.0, 1, 500, cost=1.0)             # another class (n_pix differs)
    assert est.expect(b) == 1000.0


def test_sjf_aging_admits_a_starved_scan():
    """A large scan overtaken by a stream of small ones goes first once it has
    waited max_wait seconds."""
    srv, be = make(budget=10 ** 6, policy="sjf", work_cap=1.0, max_wait=0.05, chunk=4,
                   estimate=StepEstimate(prior={1e-4: 1000, 1e-3: 4}))
    big = req(0, 0.0, 1, 40, cost=1.0, tol=1e-4)
    small = [req(1 + i, 0.0, 1, 4, cost=0.5, tol=1e-3) for i in range(60)]
    srv.run([big] + small)
    pos = be.order.index(0)
    # 4 ms per chunk, 2 small scans of 4 steps per chunk: 50 ms is ~25 chunks
    assert 0 < pos < 60
    srv2, be2 = make(budget=10 ** 6, policy="sjf", work_cap=1.0, max_wait=1e9, chunk=4,
                     estimate=StepEstimate(prior={1e-4: 1000, 1e-3: 4}))
    srv2.run([big] + small)
    assert be2.order.index(0) == 60               # without aging it goes last


def test_policy_is_checked():
    with pytest.raises(ValueError):
        Server(None, 1, policy="lifo")
