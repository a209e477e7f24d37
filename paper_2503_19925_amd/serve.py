"""Continuous-batching request loop for EXACT reconstructions.

Requests (scans with their own geometry, spectrum, counts and tolerance)
arrive over time.  The loop keeps every admitted scan's counts and iterate
resident on the device and advances all admitted scans together, a few
extragradient steps at a time, in one exact_batch.  Between those chunks it
retires scans that have stopped (copying the reconstruction to the host and
freeing their memory) and admits waiting ones, so work of requests that
arrive while others run overlaps on the device.

Admission has two limits and an order:

* memory: the sum of the admitted scans' device footprints (library state +
  the iterate and the counts) stays within an HBM budget;
* work in flight (policy "sjf"): the admitted scans' summed cost of one
  extragradient step (about the nonzeros of their projectors) stays within
  `work_cap`, a few times what fills the GPU, so the GPU stays busy while
  a scan's steps do not slow down by sharing it with every other scan;
* order (policy "sjf"): the waiting scan with the least expected work goes
  first (shortest job first): expected steps to its tolerance (the mean of
  finished scans of the same class, a prior before any) times its step cost.
  A scan that has waited `max_wait` seconds goes ahead of every younger one,
  so a large scan is not starved by a stream of small ones.

Policy "fcfs" admits in arrival order with no overtaking and no work cap
(every scan that fits in memory runs at once).

The step size is Theorem 2's rule (paper Sec. 2.1), computed in the library:
lambda_max(A^T A / n) is computed once per geometry (exact_step_size) and
handed to exact_batch_add, which forms gamma; each scan's iterates are
bitwise those of a solo exact_solve with the same step size.

The scheduler is host logic over a small backend interface (GpuBackend
below); tests drive it with a fake backend on the CPU.
"""
from dataclasses import dataclass, field
import time

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    problem: object         # synth.Problem: sizes, mu, I, y (host)
    tol: float
    max_iters: int = 20000


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    iters: int
    resid: float
    status: int             # 1 finished, 2 stopped at max_iters
    gamma: float
    x: np.ndarray = field(default=None, repr=False)

    @property
    def latency(self):
        return self.finished - self.arrival

    @property
    def queued(self):
        return self.admitted - self.arrival


def step_cost(P):
    """Relative cost of one extragradient step of a scan: its projectors'
    work, about views x bins x image side (the Joseph matrix has about 1.3 N
    nonzeros per ray), in units of 1e6."""
    return P.n_views * P.n_bins * P.n_pix * 1e-6


def scan_class(req):
    """Scans whose iteration counts are pooled for the step estimate."""
    P = req.problem
    return (P.n_pix, P.n_views, P.n_bins, getattr(P, "I0", None), req.tol)


class GpuBackend:
    """exact_batch on the current HIP device; owns the scans' x and y."""

    def __init__(self, hbm_budget_bytes, capacity=256, power_iters=100, keep_x=True):
        import torch
        from . import exact
        self.torch, self.exact = torch, exact
        self.batch = exact.Batch(hbm_budget_bytes, capacity)
        self.power_iters = power_iters
        self.keep_x = keep_x
        self.geoms, self.lams, self.live = {}, {}, {}

    def _geometry(self, P):
        key = (P.n_pix, P.n_views, P.n_bins, P.pixel_cm, P.bin_cm, P.half_turns)
        if key not in self.geoms:
            g = self.exact.Geometry(P.n_pix, P.n_views, P.n_bins, P.pixel_cm, P.bin_cm, P.half_turns)
            self.geoms[key] = g
            self.lams[key], _ = self.exact.exact_step_size(g, None, None, self.power_iters)
        return self.geoms[key], self.lams[key]

    def footprint(self, P):
        return (self.exact.exact_run_footprint(P.n_pix, P.n_views, P.n_bins)
                + 4 * P.d + 4 * P.Wn * P.n)

    def add(self, req):
        P = req.problem
        g, lam = self._geometry(P)
        dev = self.torch.device("cuda")
        y = self.torch.as_tensor(np.ascontiguousarray(P.y, dtype=np.float32), device=dev)
        x = self.torch.zeros(P.d, device=dev)
        slot = self.batch.add(g, P.mu, P.I, y, x, lambda_hat=lam, max_iters=req.max_iters,
                              tol=req.tol)
        self.live[slot] = (x, y)
        return slot, self.batch.poll(slot)[1]["gamma"]

    def step(self, n):
        self.batch.step(n)
        return self.batch.sync()

    def poll(self, slot):
        return self.batch.poll(slot)

    def retire(self, slot):
        x, _ = self.live.pop(slot)
        out = x.cpu().numpy() if self.keep_x else None
        self.batch.remove(slot)
        return out

    def close(self):
        self.batch.close()
        for g in self.geoms.values():
            g.close()
        self.geoms.clear()


class StepEstimate:
    """Expected steps to tolerance per scan class: the mean over finished
    scans of the class, else `prior` (per tolerance, else `default`)."""

    def __init__(self, prior=None, default=1000.0):
        self.prior = dict(prior or {})
        self.default = float(default)
        self.sum, self.cnt = {}, {}

    def expect(self, req):
        c = scan_class(req)
        if self.cnt.get(c):
            return self.sum[c] / self.cnt[c]
        return float(self.prior.get(req.tol, self.default))

    def record(self, req, iters):
        c = scan_class(req)
        self.sum[c] = self.sum.get(c, 0.0) + iters
        self.cnt[c] = self.cnt.get(c, 0) + 1


class Server:
    """Admission by footprint and policy, continuous batching, retirement.

    run(requests) plays the arrival times against `clock` (seconds); with
    realtime=False the clock jumps to the next arrival when the device is
    idle instead of sleeping.  policy "sjf" (default) or "fcfs" as in the
    module docstring; work_cap in step_cost units (None: no cap); max_wait
    in seconds."""

    def __init__(self, backend, hbm_budget_bytes, chunk_steps=8, realtime=True,
                 clock=time.perf_counter, on_done=None, policy="sjf", work_cap=None,
                 max_wait=10.0, estimate=None, cost=step_cost):
        if policy not in ("sjf", "fcfs"):
            raise ValueError("policy must be 'sjf' or 'fcfs'")
        self.on_done = on_done      # called with each Result as it completes
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.chunk = int(chunk_steps)
        self.realtime = realtime
        self.clock = clock
        self.policy = policy
        self.work_cap = None if policy == "fcfs" else work_cap
        self.max_wait = float(max_wait)
        self.estimate = estimate if estimate is not None else StepEstimate()
        self.cost = cost

    def _next(self, pending, t):
        """Index in `pending` of the scan to admit next (pending is in
        arrival order)."""
        if self.policy == "fcfs":
            return 0
        if t - pending[0].arrival >= self.max_wait:
            return 0                                  # oldest, waited too long
        work = [self.estimate.expect(r) * self.cost(r.problem) for r in pending]
        return int(np.argmin(work))                   # ties: earliest arrival

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            if self.backend.footprint(r.problem) > self.budget:
                raise ValueError("request %d alone exceeds the HBM budget" % r.rid)
        pending, running, results = [], {}, []
        used, load, nxt = 0, 0.0, 0
        t0 = self.clock()
        skew = 0.0                                    # simulated-time advance
        now = lambda: self.clock() - t0 + skew        # noqa: E731
        self.peak_running = 0
        self.peak_load = 0.0
        # host-side time split: set-up of admitted scans, the chunks' steps
        # (enqueue and wait), retirement; and the number of chunks
        self.stats = {"add_s": 0.0, "step_s": 0.0, "retire_s": 0.0, "chunks": 0}
        clk = self.clock
        while nxt < len(reqs) or pending or running:
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                pending.append(reqs[nxt])
                nxt += 1
            while pending:
                i = self._next(pending, t)
                r = pending[i]
                fp = self.backend.footprint(r.problem)
                c = self.cost(r.problem)
                if used + fp > self.budget:
                    break
                if (self.work_cap is not None and running and load + c > self.work_cap):
                    break
                pending.pop(i)
                t1 = clk()
                slot, gamma = self.backend.add(r)
                self.stats["add_s"] += clk() - t1
                running[slot] = (r, now(), fp, gamma, c)
                used += fp
                load += c
            self.peak_running = max(self.peak_running, len(running))
            self.peak_load = max(self.peak_load, load)
            if not running:
                if nxt < len(reqs):
                    wait = reqs[nxt].arrival - now()
                    if wait > 0:
                        if self.realtime:
                            time.sleep(wait)
                        else:
                            skew += wait
                continue
            t1 = clk()
            self.backend.step(self.chunk)
            self.stats["step_s"] += clk() - t1
            self.stats["chunks"] += 1
            for slot in list(running):
                status, info = self.backend.poll(slot)
                if status == 0:
                    continue
                r, admitted, fp, gamma, c = running.pop(slot)
                t1 = clk()
                x = self.backend.retire(slot)
                self.stats["retire_s"] += clk() - t1
                used -= fp
                load -= c
                self.estimate.record(r, info["iters"])
                results.append(Result(r.rid, r.arrival, admitted, now(), info["iters"],
                                       info["resid"], status, gamma, x))
                if self.on_done:
                    self.on_done(results[-1])
            if not running:
                load = 0.0                            # no drift from float sums
        return sorted(results, key=lambda z: z.rid)


def fcfs_latencies(arrivals, service):
    """Arrival-to-finish times of requests served one at a time in arrival
    order by a single server: request i starts when it has arrived and
    request i - 1 has finished, and takes service[i].  Returns (latencies,
    finish time of the last)."""
    finish, lat = float("-inf"), []
    for a, s in sorted(zip(arrivals, service), key=lambda z: z[0]):
        finish = max(a, finish) + s
        lat.append(finish - a)
    return lat, finish


def summarize(results, duration=None):
    """p50/p99 time-to-tolerance (arrival to result on the host), the
    queueing share, and reconstructions per second over the stream."""
    lat = np.array([r.latency for r in results])
    q = np.array([r.queued for r in results])
    first = min(r.arrival for r in results)
    last = max(r.finished for r in results)
    span = duration if duration is not None else last - first
    i99 = int(np.argsort(lat)[min(len(lat) - 1, int(np.ceil(0.99 * len(lat))) - 1)])
    return {"requests": len(results),
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()),
            "mean_queue_s": float(q.mean()),
            "p99_queue_share": float(q[i99] / lat[i99]) if lat[i99] > 0 else 0.0,
            "recon_per_s": len(results) / span if span > 0 else float("inf"),
            "capped": int(sum(1 for r in results if r.status == 2)),
            "mean_iters": float(np.mean([r.iters for r in results]))}
