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

Prints one JSON line: EG iterations/s (value), projector rays/s, the
back-projector's algorithmic-bytes roofline fraction (HIP events), and the
CPU oracle timed on a bounded sample of the same workload.
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
HBM_PEAK_GBS = 8000.0


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


def cpu_baseline(P, gamma, steps):
    """The oracle, untuned, on a bounded sample: `steps` EG iterations of the
    same workload from x = 0 with the same step size, one thread."""
    import numpy as np
    from oracle import build as oracle_build
    from oracle import oracle as ora
    if not os.path.exists(oracle_build.LIB):
        oracle_build.build()
    go = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    t0 = time.perf_counter()
    ora.eg(go, P.mu, P.I, P.y.astype(np.float64), np.zeros(P.d), gamma, steps)
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "EG iters/s", "cores": 1, "kind": "oracle",
            "sample": "%d EG steps of solve_512 from x=0 (float64 C oracle, one thread, "
                      "%.1f s)" % (steps, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--proj-reps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="EG steps of the CPU oracle baseline (0 to skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_19925_amd import exact, synth

    exact.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = synth.config_problem("solve_512", with_truth=False)
    log("workload solve_512: N=%d V=%d B=%d K=%d Wn=%d" % (P.n_pix, P.n_views, P.n_bins, P.K, P.Wn))
    g = exact.Geometry(P.n_pix, P.n_views, P.n_bins)
    y = torch.as_tensor(P.y, device=dev)
    x = torch.zeros(g.d, device=dev)

    # set-up (untimed): step size by power iteration, resident state, graph
    solver = exact.Solver(g, P.mu, P.I, y, x, max_iters=args.warmup + args.steps, tol=0.0)
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
    solver.close()
    if info["iters"] != args.warmup + args.steps:
        raise RuntimeError("solver ran %d steps, expected %d" % (info["iters"], args.warmup + args.steps))
    log("timed %d steps: %.4f ms/step (events), %.4f ms/step (wall)" % (
        args.steps, ms_step, 1e3 * wall / args.steps))

    # projector throughput and the back-projector's roofline
    nnz = exact.exact_count_nonzeros(g)
    r = torch.randn(g.n, device=dev)
    img = torch.empty(g.d, device=dev)
    s = torch.empty(g.n, device=dev)
    xb = torch.rand(g.d, device=dev)
    t_back = event_time_ms(lambda: exact.exact_backproject(g, r, img), args.proj_reps, torch)
    t_fwd = event_time_ms(lambda: exact.exact_forward(g, xb, s), args.proj_reps, torch)
    bytes_back = 4.0 * nnz + 4.0 * g.n + 4.0 * g.d
    achieved = bytes_back / (t_back * 1e-3) / 1e9
    log("nnz %d; back %.4f ms, forward(+transpose) %.4f ms" % (nnz, t_back, t_fwd))

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
        "config": {"workload": "solve_512: 512x512 image (20 random ellipses), 180 views over "
                               "180 deg, 725 bins, 30 energy bins, 3 windows, I0=1e4 Poisson",
                   "n_pix": P.n_pix, "n_views": P.n_views, "n_bins": P.n_bins,
                   "n_energies": P.K, "n_windows": P.Wn, "parallelism": "single GPU"},
        "forward_grays": g.n / (t_fwd * 1e-3) / 1e9,
        "back_grays": g.n / (t_back * 1e-3) / 1e9,
        "forward_ms": t_fwd,
        "back_ms": t_back,
        "nnz": nnz,
        "roofline": {"kernel": "k_back", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
        "cpu_baseline": base,
    }
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
