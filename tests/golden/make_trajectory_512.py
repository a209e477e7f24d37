"""Writes tests/golden/trajectory_solve_512.txt: the CPU oracle's EXACT run on
the solve_512 workload (512x512, 180 views, 725 bins, K=30, Wn=3, I0=1e4;
synthetic seeds 201/202), 500 steps from x = 0.

Calls only the oracle (and the seeded input generator).  The step size is
Theorem 2's gamma = 1/(4 lambda_max(A^T A/n) sum_k J_k mu_k) with lambda_max
from the oracle's power iteration.  Stored: gamma, lambda, the iterate's
norm, and the values of 4096 pixels drawn with a fixed seed, in double
precision; also the same run in single precision (the oracle's float build),
which states how far a float computation can drift from the double one.

Takes about half an hour per precision on one core:
    python tests/golden/make_trajectory_512.py [f64|f32|both]
"""
import os
import sys
import time
from multiprocessing import Process

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as ora  # noqa: E402
from paper_2503_19925_amd import synth  # noqa: E402

STEPS = 500
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trajectory_solve_512.txt")
SAMPLE_SEED = 512
N_SAMPLE = 4096


def run(prec, gamma, lam, path):
    P = synth.config_problem("solve_512", with_truth=False)
    g = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    t0 = time.time()
    x, t, _ = ora.eg(g, P.mu, P.I, P.y.astype(np.float64), np.zeros(P.d), gamma, STEPS, prec=prec)
    np.save(path, x)
    print("%s: %d steps in %.0f s" % (prec, t, time.time() - t0), flush=True)


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "both"
    P = synth.config_problem("solve_512", with_truth=False)
    g = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    t0 = time.time()
    lam, it = ora.power(g, 300, 1e-9)
    gamma = ora.step_size(lam, P.mu, P.I)
    print("lambda %.12e after %d power steps (%.0f s); gamma %.12e" % (lam, it, time.time() - t0, gamma),
          flush=True)
    tmp = {p: OUT + "." + p + ".npy" for p in ("f64", "f32")}
    precs = ["f64", "f32"] if which == "both" else [which]
    procs = [Process(target=run, args=(p, gamma, lam, tmp[p])) for p in precs]
    for p in procs:
        p.start()
    for p in procs:
        p.join()
    x64 = np.load(tmp["f64"])
    rng = np.random.default_rng(SAMPLE_SEED)
    pix = np.sort(rng.choice(P.d, size=N_SAMPLE, replace=False))
    lines = ["# EXACT oracle trajectory, workload solve_512, %d steps from x = 0" % STEPS,
             "# written by tests/golden/make_trajectory_512.py (oracle only)",
             "# y checksum = sum of all counts; sample pixels drawn with seed %d" % SAMPLE_SEED,
             "steps = %d" % STEPS,
             "lambda = %.17g" % lam,
             "gamma = %.17g" % gamma,
             "y_sum = %.17g" % float(P.y.astype(np.float64).sum()),
             "x_norm = %.17g" % float(np.linalg.norm(x64))]
    if os.path.exists(tmp["f32"]):
        x32 = np.load(tmp["f32"])
        lines.append("f32_rel_l2 = %.6e" % (np.linalg.norm(x32 - x64) / np.linalg.norm(x64)))
    lines.append("# pixel value")
    lines += ["%d %.17g" % (p, x64[p]) for p in pix]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    for p in tmp.values():
        if os.path.exists(p):
            os.remove(p)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
