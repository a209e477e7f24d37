#!/usr/bin/env python3
"""EXACT benchmark on one MI355X.

Workload: solve_512 -- a 512 x 512 random-ellipse phantom (20 ellipses),
180 parallel-beam views over 180 degrees, 725 detector bins of pixel width,
30 energy bins (20-120 keV), 3 windows, I0 = 1e4 photons per ray, Poisson
counts.  One step = one full projected-extragradient iteration (two operator
evaluations: forward projection with the fused spectral residual,
back-projection, update and projection, twice; plus the double-precision
residual reduction and stop test), replayed from a captured HIP graph with
all state resident in HBM.

Prints one JSON line: EG iterations/s (value), projector rays/s, and the
roofline of the step's dominant kernel (`roofline`: whichever of the forward
with its residual epilogue and the back-projection fused with the update
takes more of the step; the other in `roofline_other`).  The kernels are
bound by VALU instruction issue (no dense contraction, and on-chip reuse
serves nearly all operand traffic), so the roofline is taken against the
VALU issue rate: the kernel's VALU lane-instructions per launch (from the
hardware counter SQ_INSTS_VALU of the committed profile when it was taken on
the library as built now, else the instruction count of its inner loop) over its average
launch duration, measured live with HIP events around back-to-back launches
on the solver's stream.  Beside it: measured HBM bytes and rate, and the
algorithmic bytes (4 B per nonzero of A), labelled as not a bound.  The CPU
oracle is timed on a bounded sample of the same workload.  More legs report
the 1024^2 workload solved to tolerance, reconstructions/s and
time-to-tolerance percentiles:

* batched: 64 uneven scans (N in {128..768}, 30-360 views, 10-64 energy
  bins, 2-4 windows; seed 401), each to natural residual 1e-4 (cap 5000
  steps), once one at a time with exact_solve and once in one batch;
  results are bitwise equal, so the accuracy is equal;
* served: the first --served requests (default 300) of a seeded Poisson
  stream at 20 requests/s (N in {256, 512, 1024}, 90/180/360 views, K = 30, Wn = 3,
  I0 in {1e3, 1e4}, tolerance 1e-3 or 1e-4), admitted by HBM footprint,
  shortest expected work first under a cap on work in flight, and batched
  continuously; time-to-tolerance runs from arrival to the result on the
  host.  Beside it the same stream served one request at a time in arrival
  order (FCFS).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EG iters/s + projector Grays/s @512²×180 views; batched p50/p99 time-to-tol"
WORKLOADS = {
    "solve_512": "solve_512: 512x512 image (20 random ellipses), 180 views over 180 deg, "
                 "725 bins, 30 energy bins, 3 windows, I0=1e4 Poisson",
    "large_1024": "large_1024: 1024x1024 image (40 random ellipses), 720 views over 180 deg, "
                  "1448 bins, 64 energy bins, 4 windows, I0=1e3 Poisson",
}
HBM_PEAK_GBS = 8000.0
# VALU issue peak: the published FP32 vector rate, 157.3 TFLOP/s = 78.6 T
# lane-operations/s (256 CUs x 4 SIMDs x one wave64 instruction per 2 cycles
# x 2.4 GHz).  Measured on MI355X, two-operand 32-bit instructions issue at
# that rate, while the three-operand FP32 FMA and the FP64 add and fract take
# 4 cycles; so for a kernel's mix this peak is an upper bound, and its
# fraction a lower bound.
VALU_PEAK_TOPS = 256 * 4 * 64 * 2.4e9 / 2 / 1e12
# VALU instructions of the inner loops, counted in their gfx950 assembly
# (Kahan steps included): per pixel and view in the gather (clamp-free
# form, which the benchmark geometry uses), per ray and line in the forward
# (two rays per lane).  Used only when no counter reading of the current
# build is committed; the counters also see the forward's lanes on lines
# their rays miss, its epilogue and loop control (about 17.7 per ray-line).
VALU_PER_PIXEL_VIEW = 14.0
VALU_PER_RAY_LINE = 10.25
KERNEL_FWD = "k_forward<true>"
KERNEL_BU = "k_back_update"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def event_time_ms(fn, reps, torch):
    """Average duration of fn() over reps calls, HIP events on the current stream."""
    st = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def host_cpu():
    """(logical CPUs this process may use, CPU model name)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


def _cpu_worker(job):
    """One process of the all-core oracle run (a fresh interpreter that
    imports only numpy and the oracle)."""
    import numpy as np
    from oracle import oracle as ora
    n_pix, n_views, n_bins, mu, I, y, gamma, steps = job
    go = ora.Geom(n_pix, n_views, n_bins)
    ora.eg(go, mu, I, y, np.zeros(n_pix * n_pix), gamma, steps)
    return steps


def cpu_baseline(P, gamma, steps, par_steps=2):
    """The oracle, untuned, on a bounded sample: `steps` EG iterations of the
    same workload from x = 0 with the same step size.  The oracle is serial
    C, so one reconstruction runs on one thread (`value`); beside it, every
    host CPU this process may use runs its own copy of the same sample
    (`par_steps` steps each, one process per CPU), which gives the host's
    aggregate oracle throughput over independent reconstructions."""
    import multiprocessing as mp
    import numpy as np
    from oracle import build as oracle_build
    from oracle import oracle as ora
    if not os.path.exists(oracle_build.LIB):
        oracle_build.build()
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    t0 = time.perf_counter()
    ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(P.d), gamma, steps)
    dt = time.perf_counter() - t0
    ncpu, model = host_cpu()
    rec = {"value": steps / dt, "unit": "EG iters/s", "cores": 1, "kind": "oracle",
           "sample": "%d EG steps of %s from x=0 (float64 C oracle, serial: one thread, "
                     "%.1f s)" % (steps, P.name, dt),
           "host_cpus": ncpu, "cpu_model": model}
    if par_steps > 0 and ncpu > 1:
        job = (P.n_pix, P.n_views, P.n_bins, np.asarray(P.mu, dtype=np.float64),
               np.asarray(P.I, dtype=np.float64), P.y.astype(np.float64), gamma, par_steps)
        ctx = mp.get_context("spawn")
        with ctx.Pool(ncpu) as pool:
            pool.map(abs, range(ncpu))                # interpreters started before timing
            t0 = time.perf_counter()
            done = sum(pool.map(_cpu_worker, [job] * ncpu, chunksize=1))
            dtp = time.perf_counter() - t0
        rec["all_cores"] = {"value": done / dtp, "unit": "EG iters/s (aggregate)", "cores": ncpu,
                            "sample": "%d processes x %d EG steps of %s, one per CPU (%.1f s)"
                                      % (ncpu, par_steps, P.name, dtp)}
    return rec


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic.json: rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a
    plain copy's reading), or None when the kernel source or its tile knobs
    have changed since the counters were taken."""
    from paper_2503_19925_amd import build as libbuild
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
        if rec.get("kernel_build_id") != libbuild.build_id():
            return None
        return rec["workloads"][workload][kernel]["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def measured_valu(workload, kernel):
    """VALU lane-instructions per launch of `kernel` (SQ_INSTS_VALU per
    dispatch x 64 lanes) from the committed counter summary
    (profiles/valu.json), or None when the kernel source or its tile knobs
    have changed since the counters were taken."""
    from paper_2503_19925_amd import build as libbuild
    path = os.path.join(ROOT, "profiles", "valu.json")
    try:
        rec = json.load(open(path))
        if rec.get("kernel_build_id") != libbuild.build_id():
            return None
        return rec["workloads"][workload][kernel]["valu_lane_instr_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def kernel_roofline(name, workload, ms, static_valu, alg_bytes):
    """The roofline record of one kernel: VALU issue (the binding unit),
    then the measured HBM traffic and the algorithmic bytes beside it."""
    valu = measured_valu(workload, name)
    src = "counters: SQ_INSTS_VALU x 64 per dispatch (profiles/valu.json)"
    if valu is None:
        valu, src = static_valu, "static: inner-loop instructions x units"
    achieved = valu / (ms * 1e-3) / 1e12
    traffic = measured_traffic(workload, name)
    rec = {"kernel": name, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
           "unit": "T VALU lane-instructions/s", "frac": achieved / VALU_PEAK_TOPS,
           "frac_at_4_cycles": 2.0 * achieved / VALU_PEAK_TOPS,
           "peak_note": "published FP32 vector rate (one wave64 instruction per 2 cycles per "
                        "SIMD); the FP64 crossing arithmetic and three-operand FMAs issue at "
                        "one per 4 cycles, against which frac_at_4_cycles is taken: the "
                        "kernel's mix bound lies between the two",
           "traffic": traffic, "ms_per_launch": ms,
           "valu_lane_instr_per_launch": valu, "valu_source": src,
           "hbm": None if traffic is None else {
               "achieved": traffic / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "algorithmic": {"bytes_per_launch": alg_bytes,
                           "GB_per_s": alg_bytes / (ms * 1e-3) / 1e9,
                           "note": "4 B per nonzero of A plus compulsory I/O; served from "
                                   "L2/L1, not a bound"}}
    return rec


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def batched_leg(count, torch, exact, synth, serial=True):
    """Same scans, one at a time and batched; wall time includes each scan's
    set-up (validation, power iteration) on both sides.  serial = False skips
    the one-at-a-time pass (for profiling the batched kernels alone); the
    serial figures and the bitwise comparison are then None."""
    tol, cap = 1e-4, 5000
    Ps = [synth.make_problem("batch%d" % i, with_truth=False, **d)
          for i, d in enumerate(synth.batch_draws(count, 401))]
    geos = [exact.Geometry(P.n_pix, P.n_views, P.n_bins) for P in Ps]
    ys = [torch.as_tensor(P.y, device="cuda") for P in Ps]
    torch.cuda.synchronize()
    log("batched leg: %d scans generated" % count)
    xs_serial, iters_serial, done_serial = [], [], []
    t0 = time.perf_counter()
    for P, g, y in (zip(Ps, geos, ys) if serial else ()):
        x = torch.zeros(g.d, device="cuda")
        info = exact.exact_solve(g, P.mu, P.I, y, x, max_iters=cap, tol=tol, check_every=32)
        if len(xs_serial) % 16 == 15:
            log("serial: %d scans done" % (len(xs_serial) + 1))
        xs_serial.append(x)
        iters_serial.append(info["iters"])
        done_serial.append(time.perf_counter() - t0)
    t_serial = time.perf_counter() - t0 if serial else None
    if serial:
        log("serial: %.2f s" % t_serial)
    footprint = sum(exact.exact_run_footprint(P.n_pix, P.n_views, P.n_bins) for P in Ps)
    xs = [torch.zeros(g.d, device="cuda") for g in geos]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = exact.Batch(footprint + (1 << 20), capacity=count)
    slots = [b.add(g, P.mu, P.I, y, x, max_iters=cap, tol=tol) for P, g, y, x in zip(Ps, geos, ys, xs)]
    done_at = {}
    while len(done_at) < count:
        b.step(32)
        b.sync()
        now = time.perf_counter() - t0
        for s in slots:
            if s not in done_at and b.poll(s)[0] != exact.RUNNING:
                done_at[s] = now
    t_batch = time.perf_counter() - t0
    stats = [b.poll(s) for s in slots]
    b.close()
    log("batched: %.2f s" % t_batch)
    same = (all(st[1]["iters"] == it for st, it in zip(stats, iters_serial)) and
            all(torch.equal(a, c) for a, c in zip(xs, xs_serial))) if serial else None
    capped = sum(1 for st in stats if st[0] == exact.CAPPED)
    for g in geos:
        g.close()
    t_done = [done_at[s] for s in slots]
    return {"scans": count, "tol": tol, "max_iters": cap,
            "serial_recon_per_s": count / t_serial if serial else None,
            "batched_recon_per_s": count / t_batch,
            "speedup": t_serial / t_batch if serial else None,
            "bitwise_equal_to_serial": bool(same) if serial else None,
            "capped": capped, "mean_iters": sum(st[1]["iters"] for st in stats) / count,
            "batched_p50_s": pct(t_done, 50), "batched_p99_s": pct(t_done, 99),
            "serial_p50_s": pct(done_serial, 50) if serial else None,
            "serial_p99_s": pct(done_serial, 99) if serial else None}


def tv_leg(P, gamma, steps, torch, exact, synth):
    """The constraint set of the paper's experiments (TV ball and orthant) at
    the workload's size: one projection of a noisy copy of the phantom onto
    {TV <= TV(phantom)} and the orthant, and `steps` EG steps over that set
    from the same start.  The TV bound is the phantom's own (the paper's
    oracle bound)."""
    import numpy as np
    N = P.n_pix
    truth = synth.phantom_image(P.ell, N, P.pixel_cm)
    tau = exact.exact_tv_norm(torch.as_tensor(truth.astype(np.float32), device="cuda"))
    rng = np.random.default_rng(7)
    z = np.maximum(0, truth + rng.normal(scale=0.2, size=truth.size)).astype(np.float32)
    zt = torch.as_tensor(z, device="cuda")
    out = torch.empty_like(zt)
    info = exact.exact_project_tv(zt, tau, out)
    fgp_steps = info["solves"] * 100
    per_step_ms = info["ms"] / max(fgp_steps, 1)
    res = {"tau": tau, "projection_ms": info["ms"], "rounds": info["rounds"],
           "prox_solves": info["solves"], "ms_per_fgp_step": per_step_ms,
           "fgp_note": "wall time of the projection per FGP step (searches, Dykstra rounds and "
                       "launch gaps included); a launch takes 8 steps with the state in LDS, so "
                       "HBM moves 36 B per pixel per launch, not per step: the steps are bound "
                       "by the workgroups' arithmetic and barriers, not by HBM"}
    log("tv projection at %d^2: %.1f ms, %d rounds, %d solves" % (N, info["ms"], info["rounds"],
                                                                  info["solves"]))
    if steps > 0:
        # `steps` EG steps from the noisy start, and the same run cut at its
        # first two steps (deterministic, so the difference is the cost of
        # the later steps); the first steps carry the searches' cold start
        g = exact.Geometry(P.n_pix, P.n_views, P.n_bins)
        y = torch.as_tensor(P.y, device="cuda")
        runs = {}
        for n in sorted({min(2, steps), steps}):
            x = torch.as_tensor(z, device="cuda")
            runs[n] = exact.exact_solve_tv(g, P.mu, P.I, y, x, tau, gamma=gamma, max_iters=n)
        g.close()
        sinfo, tinfo = runs[steps]
        res.update({"eg_steps": sinfo["iters"], "ms_per_eg_step": sinfo["ms"] / max(sinfo["iters"], 1),
                    "eg_prox_solves": tinfo["solves"], "tv_after": tinfo["tv"]})
        s2, t2 = runs[min(2, steps)]
        res["first_steps"] = {"steps": s2["iters"], "ms_per_eg_step": s2["ms"] / max(s2["iters"], 1),
                              "prox_solves": t2["solves"]}
        if steps > 2:
            k = sinfo["iters"] - s2["iters"]
            res["later_steps"] = {"steps": k, "ms_per_eg_step": (sinfo["ms"] - s2["ms"]) / max(k, 1),
                                  "prox_solves_per_step": (tinfo["solves"] - t2["solves"]) / max(k, 1)}
        log("tv EG: %d steps, %.1f ms/step, %d solves (first %d steps %.1f ms/step)" % (
            sinfo["iters"], res["ms_per_eg_step"], tinfo["solves"], s2["iters"],
            res["first_steps"]["ms_per_eg_step"]))
    return res


def dense_leg(d, mult, steps, torch, exact):
    """The Gaussian measurement model at scale: A is (mult d) x d standard
    normal float32, drawn on the device with a seeded generator, x* of norm 3,
    noiseless monochromatic counts y = exp(-max(A x*, 0)) (the set-up of the
    paper's Gaussian experiment, larger).  Times `steps` EG steps with
    gamma = 0.25; each step evaluates F twice, each evaluation reads A once."""
    n = mult * d
    gen = torch.Generator(device="cuda")
    gen.manual_seed(601)
    A = torch.randn(n, d, device="cuda", generator=gen)
    xs = torch.randn(d, device="cuda", generator=gen)
    xs *= 3.0 / torch.linalg.vector_norm(xs)
    y = torch.exp(-torch.clamp(A @ xs, min=0.0))
    x = torch.zeros(d, device="cuda")
    exact.exact_dense_solve(A, [1.0], [1.0], y, x, gamma=0.25, max_iters=2)   # warm-up
    x.zero_()
    torch.cuda.synchronize()
    info = exact.exact_dense_solve(A, [1.0], [1.0], y, x, gamma=0.25, max_iters=steps,
                                   check_every=steps)
    ms_step = info["ms"] / steps
    bytes_f = 4.0 * n * d
    achieved = 2 * bytes_f / (ms_step * 1e-3) / 1e9
    err = float(torch.linalg.vector_norm(x - xs) / 3.0)
    log("dense %d x %d: %.3f ms per EG step (%.1f GB/s over two reads of A)" % (
        n, d, ms_step, achieved))
    del A
    return {"n": n, "d": d, "steps": steps, "ms_per_step": ms_step,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "note": "4 n d bytes per F evaluation, two per step; wall time of "
                                 "the call, set-up included"},
            "rel_error_after": err}


def fcfs_one_at_a_time(reqs, torch, exact, power_iters=100):
    """The same requests served one at a time in arrival order (first come,
    first served) on the same GPU: each is solved alone by exact_solve with
    its own step size, tolerance and cap (so the reconstructions equal the
    served ones bit for bit), its service time measured on the wall clock
    (counts upload + solve; geometry and lambda_max cached per shape as the
    server does), and the queue formed from the stream's arrival times."""
    import numpy as np
    from paper_2503_19925_amd.serve import fcfs_latencies
    order = sorted(reqs, key=lambda r: (r.arrival, r.rid))
    geoms, svc = {}, []
    for r in order:
        P = r.problem
        key = (P.n_pix, P.n_views, P.n_bins, P.pixel_cm, P.bin_cm, P.half_turns)
        if key not in geoms:
            g = exact.Geometry(P.n_pix, P.n_views, P.n_bins, P.pixel_cm, P.bin_cm, P.half_turns)
            geoms[key] = (g, exact.exact_step_size(g, None, None, power_iters)[0])
        g, lam = geoms[key]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = torch.as_tensor(np.ascontiguousarray(P.y, dtype=np.float32), device="cuda")
        x = torch.zeros(P.d, device="cuda")
        exact.exact_solve(g, P.mu, P.I, y, x, lambda_hat=lam, max_iters=r.max_iters, tol=r.tol)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t0)
    for g, _ in geoms.values():
        g.close()
    lats, finish = fcfs_latencies([r.arrival for r in order], svc)
    span = finish - order[0].arrival
    return {"p50_s": pct(lats, 50), "p99_s": pct(lats, 99),
            "recon_per_s": len(reqs) / span, "service_s_total": float(sum(svc)),
            "note": "queue simulated from the measured solo solve times and the arrivals"}


def large_leg(tol, torch, exact, synth, reps):
    """The large low-dose workload (1024^2 image, 720 views x 1448 bins,
    K = 64, Wn = 4, I0 = 1e3): the step's kernel durations and projector
    rays/s, and a solve from x = 0 to natural residual `tol` (cap 20000
    steps), timed on the wall clock around exact_solve (set-up included)."""
    import numpy as np
    P = synth.config_problem("large_1024", with_truth=False)
    log("large_1024: generated")
    g = exact.Geometry(P.n_pix, P.n_views, P.n_bins)
    y = torch.as_tensor(P.y, device="cuda")
    x = torch.zeros(g.d, device="cuda")
    sv = exact.Solver(g, P.mu, P.I, y, x, max_iters=4, tol=0.0)
    sv.step(4)
    kms = sv.time_kernels(max(2, reps // 4))
    _, info = sv.poll()
    sv.close()
    st = torch.cuda.current_stream()
    x.zero_()
    sv = exact.Solver(g, P.mu, P.I, y, x, gamma=info["gamma"], max_iters=22, tol=0.0)
    sv.step(2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    sv.step(20)
    e1.record(st)
    e1.synchronize()
    sv.close()
    ms_step = e0.elapsed_time(e1) / 20
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = exact.exact_solve(g, P.mu, P.I, y, x, max_iters=20000, tol=tol, check_every=32)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    fwd_ms, bu_ms = (kms[0] + kms[2]) / 2, (kms[1] + kms[3]) / 2
    log("large_1024: %.4f ms/step; to %.0e in %d steps, %.2f s" % (ms_step, tol, it["iters"], wall))
    return {"workload": WORKLOADS["large_1024"], "ms_per_step": ms_step,
            "EG_iters_per_s": 1e3 / ms_step, "kernel_ms": dict(zip(exact.PHASE_NAMES, kms)),
            "forward_grays": g.n / (fwd_ms * 1e-3) / 1e9, "back_grays": g.n / (bu_ms * 1e-3) / 1e9,
            "to_tol": {"tol": tol, "iters": it["iters"], "resid": it["resid"],
                       "converged": it["converged"], "seconds": wall,
                       "seconds_in_call": it["ms"] / 1e3, "gamma": it["gamma"]}}


def served_leg(count, torch, exact, synth, serial=True, policy="sjf", work_cap=2500.0,
               max_wait=10.0, admit_all=False, chunk=16):
    from paper_2503_19925_amd.serve import GpuBackend, Request, Server, summarize
    stream = synth.served_stream(300, 20.0, 501)[:count]
    reqs = [Request(q, s["arrival"], synth.make_problem("req%d" % q, with_truth=False,
                                                        **s["params"]), s["tol"], 20000)
            for q, s in enumerate(stream)]
    log("served leg: %d requests generated" % count)
    budget = 64 << 30

    def progress(r):
        log("served: request %d done (%d steps, %.2f s after arrival)" % (r.rid, r.iters, r.latency))

    def play(pol, cap):
        be = GpuBackend(budget, capacity=max(8, count), keep_x=False)
        srv = Server(be, budget, chunk_steps=chunk, on_done=progress, policy=pol, work_cap=cap,
                     max_wait=max_wait)
        res = srv.run(reqs)
        be.close()
        out = summarize(res)
        out.update({"policy": pol, "work_cap": cap, "peak_running": srv.peak_running,
                    "host": srv.stats})
        if pol == "sjf":
            out["max_wait_s"] = max_wait
        return out

    s = play(policy, work_cap)
    s["offered_req_per_s"] = (count - 1) / (reqs[-1].arrival - reqs[0].arrival)
    if admit_all:
        a = play("fcfs", None)
        log("served admit-all (FCFS, no cap): p50 %.2f s, p99 %.2f s, %.2f recon/s"
            % (a["p50_s"], a["p99_s"], a["recon_per_s"]))
        s["admit_all_fcfs"] = a
    if serial:
        f = fcfs_one_at_a_time(reqs, torch, exact)
        log("served one at a time (FCFS): p50 %.2f s, p99 %.2f s, %.2f recon/s"
            % (f["p50_s"], f["p99_s"], f["recon_per_s"]))
        s["fcfs_one_at_a_time"] = f
    return s


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--proj-reps", type=int, default=50)
    ap.add_argument("--kernel-reps", type=int, default=20,
                    help="back-to-back launches per step kernel for its average duration")
    ap.add_argument("--cpu-steps", type=int, default=8,
                    help="EG steps of the CPU oracle baseline (0 to skip)")
    ap.add_argument("--batch", type=int, default=64, help="scans in the batched leg (0 to skip)")
    ap.add_argument("--dense-steps", type=int, default=50,
                    help="EG steps of the dense Gaussian-model leg (0 skips it)")
    ap.add_argument("--tv-steps", type=int, default=8,
                    help="EG steps over the TV ball and orthant after one projection "
                         "(-1 skips the TV leg)")
    ap.add_argument("--background-steps", type=int, default=100,
                    help="timed steps of the workload with known materials (0 to skip)")
    ap.add_argument("--served", type=int, default=300,
                    help="requests in the served leg (0 to skip)")
    ap.add_argument("--batch-serial", type=int, default=1,
                    help="0: skip the batched leg's one-at-a-time pass (profiling)")
    ap.add_argument("--served-serial", type=int, default=1,
                    help="also serve the stream one request at a time (0 to skip)")
    ap.add_argument("--served-policy", default="sjf", choices=("sjf", "fcfs"),
                    help="admission order of the served leg")
    ap.add_argument("--served-cap", type=float, default=2500.0,
                    help="work in flight of the served leg (step-cost units; <= 0: no cap)")
    ap.add_argument("--served-max-wait", type=float, default=10.0,
                    help="seconds after which a waiting request goes first")
    ap.add_argument("--served-admit-all", type=int, default=0,
                    help="also serve the stream admitting every request at once (FCFS)")
    ap.add_argument("--large-to-tol", type=float, default=1e-4,
                    help="solve the 1024^2 workload from x=0 to this natural residual "
                         "(0 to skip)")
    ap.add_argument("--workload", default="solve_512", choices=sorted(WORKLOADS),
                    help="single-scan workload of the main line")
    ap.add_argument("--to-tol", type=float, default=0.0,
                    help="also solve the workload from x=0 to this natural residual")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run a plain device copy of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_19925_amd import exact, synth

    exact.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = synth.config_problem(args.workload, with_truth=False)
    log("workload %s: N=%d V=%d B=%d K=%d Wn=%d" % (P.name, P.n_pix, P.n_views, P.n_bins, P.K, P.Wn))
    if args.calibrate_copy_mb > 0:
        src = torch.ones(args.calibrate_copy_mb << 18, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d MiB" % args.calibrate_copy_mb)
        del src, dst
    g = exact.Geometry(P.n_pix, P.n_views, P.n_bins)
    y = torch.as_tensor(P.y, device=dev)
    x = torch.zeros(g.d, device=dev)

    # set-up (outside the timed region, reported): step size by power
    # iteration (100 products with A^T A), resident state, graph capture
    torch.cuda.synchronize()
    t_set = time.perf_counter()
    solver = exact.Solver(g, P.mu, P.I, y, x, max_iters=args.warmup + args.steps, tol=0.0)
    setup_ms = 1e3 * (time.perf_counter() - t_set)
    torch.cuda.synchronize()
    t_set = time.perf_counter()
    lam_only, _ = exact.exact_step_size(g, None, None, 100)
    power_ms = 1e3 * (time.perf_counter() - t_set)
    log("set-up %.1f ms (power iteration alone %.1f ms)" % (setup_ms, power_ms))
    solver.step(args.warmup)
    torch.cuda.synchronize()
    _, info_w = solver.poll()
    log("warmup done: %d steps, gamma %.4e, lambda %.4e" % (info_w["iters"], info_w["gamma"],
                                                          info_w["lambda_hat"]))

    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    solver.step(args.steps)
    e1.record(st)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    done, info = solver.poll()
    if info["iters"] != args.warmup + args.steps:
        raise RuntimeError("solver ran %d steps, expected %d" % (info["iters"], args.warmup + args.steps))
    log("timed %d steps: %.4f ms/step (events), %.4f ms/step (wall)" % (
        args.steps, ms_step, 1e3 * wall / args.steps))
    # each kernel of the step launched kernel_reps times back to back between
    # two HIP events on the solver's stream: average duration per launch
    kms = solver.time_kernels(args.kernel_reps)
    solver.close()
    log("kernel ms: " + ", ".join("%s %.4f" % (n, t) for n, t in zip(exact.PHASE_NAMES, kms)))

    # standalone projector calls (each pads or weighs its input first)
    nnz = exact.exact_count_nonzeros(g)
    r = torch.randn(g.n, device=dev)
    img = torch.empty(g.d, device=dev)
    s = torch.empty(g.n, device=dev)
    xb = torch.rand(g.d, device=dev)
    t_back = event_time_ms(lambda: exact.exact_backproject(g, r, img), args.proj_reps, torch)
    t_fwd = event_time_ms(lambda: exact.exact_forward(g, xb, s), args.proj_reps, torch)
    log("nnz %d; exact_backproject %.4f ms, exact_forward %.4f ms (calls)" % (nnz, t_back, t_fwd))
    fwd_ms = (kms[0] + kms[2]) / 2
    bu_ms = (kms[1] + kms[3]) / 2
    # algorithmic bytes (4 B per nonzero of A plus compulsory I/O): the
    # forward reads x per nonzero, Y per ray and writes r; the
    # back-projection + update gathers r per nonzero, reads r once and x,
    # writes z to the padded pair (and to x in the full step)
    bytes_fwd = 4.0 * nnz + 8.0 * g.d + 8.0 * g.n
    bytes_bu = 4.0 * nnz + 4.0 * g.n + 14.0 * g.d
    roof_fwd = kernel_roofline(KERNEL_FWD, args.workload, fwd_ms,
                               VALU_PER_RAY_LINE * nnz / 2.0, bytes_fwd)
    roof_back = kernel_roofline(KERNEL_BU, args.workload, bu_ms,
                                VALU_PER_PIXEL_VIEW * g.d * P.n_views, bytes_bu)
    # the dominant kernel: the one that takes more of the step (two launches each)
    roof_dominant, roof_other = ((roof_fwd, roof_back) if fwd_ms >= bu_ms
                                 else (roof_back, roof_fwd))
    log("roofline %s: %.3f of VALU issue (%s)" % (roof_dominant["kernel"], roof_dominant["frac"],
                                                 roof_dominant["valu_source"].split(":")[0]))

    large = None
    if args.large_to_tol > 0 and args.workload != "large_1024":
        large = large_leg(args.large_to_tol, torch, exact, synth, args.kernel_reps)

    to_tol = None
    if args.to_tol > 0:
        xt = torch.zeros(g.d, device=dev)
        info_t = exact.exact_solve(g, P.mu, P.I, y, xt, max_iters=20000, tol=args.to_tol,
                                   check_every=32)
        to_tol = {"tol": args.to_tol, "iters": info_t["iters"], "resid": info_t["resid"],
                  "converged": info_t["converged"], "seconds": info_t["ms"] / 1e3}
        log("to tolerance %.0e: %d steps, %.2f s" % (args.to_tol, info_t["iters"], info_t["ms"] / 1e3))

    # the same workload with known materials (the appendix's reparametrised
    # model): one more per-ray input in the residual epilogue
    background = None
    if args.background_steps > 0:
        Pb = synth.with_background(P)
        bgt = torch.as_tensor(Pb.bg.astype("float32"), device=dev)
        yb = torch.as_tensor(Pb.y, device=dev)
        xb0 = torch.zeros(g.d, device=dev)
        sb = exact.Solver(g, Pb.mu, Pb.I, yb, xb0, gamma=info["gamma"], tol=0.0,
                          max_iters=10 + args.background_steps, background=bgt)
        sb.step(10)
        torch.cuda.synchronize()
        e0.record(st)
        sb.step(args.background_steps)
        e1.record(st)
        e1.synchronize()
        sb.close()
        ms_bg = e0.elapsed_time(e1) / args.background_steps
        background = {"ms_per_step": ms_bg, "EG_iters_per_s": 1000.0 / ms_bg,
                      "relative_to_plain": ms_bg / ms_step}
        log("known background: %.4f ms/step" % ms_bg)

    tv = None
    if args.tv_steps >= 0:
        Pt = synth.config_problem(args.workload, with_truth=False)
        tv = tv_leg(Pt, info["gamma"], args.tv_steps, torch, exact, synth)

    dense = dense_leg(4096, 20, args.dense_steps, torch, exact) if args.dense_steps > 0 else None

    batched = (batched_leg(args.batch, torch, exact, synth, serial=args.batch_serial > 0)
               if args.batch > 0 else None)
    served = (served_leg(args.served, torch, exact, synth, serial=args.served_serial > 0,
                         policy=args.served_policy,
                         work_cap=args.served_cap if args.served_cap > 0 else None,
                         max_wait=args.served_max_wait, admit_all=args.served_admit_all > 0)
              if args.served > 0 else None)
    if served:
        log("served: p50 %.2f s, p99 %.2f s, %.2f recon/s" % (served["p50_s"], served["p99_s"],
                                                             served["recon_per_s"]))

    base = None
    if args.cpu_steps > 0:
        log("cpu baseline: %d oracle EG steps" % args.cpu_steps)
        base = cpu_baseline(P, info["gamma"], args.cpu_steps)

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_step,
        "unit": "EG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "n_pix": P.n_pix, "n_views": P.n_views, "n_bins": P.n_bins,
                   "n_energies": P.K, "n_windows": P.Wn, "parallelism": "single GPU"},
        "forward_grays": g.n / (fwd_ms * 1e-3) / 1e9,
        "back_grays": g.n / (bu_ms * 1e-3) / 1e9,
        "grays_note": "rays per second of the step's kernels (forward + residual; "
                      "back-projection + update), average launch durations",
        "call_forward_grays": g.n / (t_fwd * 1e-3) / 1e9,
        "call_back_grays": g.n / (t_back * 1e-3) / 1e9,
        "call_forward_ms": t_fwd,
        "call_back_ms": t_back,
        "nnz": nnz,
        "kernel_ms": dict(zip(exact.PHASE_NAMES, kms)),
        "setup_ms": setup_ms,
        "power_iteration_ms": power_ms,
        "roofline": roof_dominant,
        "roofline_other": roof_other,
        "large_1024": large,
        "to_tol": to_tol,
        "background": background,
        "tv_ball": tv,
        "dense_gaussian": dense,
        "cpu_baseline": base,
        "batched": batched,
        "served": served,
    }
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
