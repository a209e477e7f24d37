"""Writes tests/golden/large_1024.txt: the CPU oracle on the large low-dose
workload large_1024 (1024x1024, 720 views, 1448 bins, K=64, Wn=4, I0=1e3;
synthetic seeds 301/302).

Calls only the oracle (and the seeded input generator).  Stored, in double
precision:

* the operator (paper Sec. 1.2, eq. operator) at x = float32(0.9 x_true):
  F at 4096 pixels and r at 4096 rays drawn with a fixed seed, each with its
  per-element scale ((1/n) A^T (Y + m) for F, Y + m for r, m the model
  counts), so a test can apply the per-element parity bar;
* EXACT (eq. extragrad-method) from x = 0 for STEPS steps with Theorem 2's
  step size taken on an upper bound of lambda_max(A^T A / n): the product of
  A's largest row sum and largest column sum, over n (a smaller step than
  the power-iteration one, and a valid one for the theorem); the iterate at
  the same 4096 pixels and its norm.  The same run in the oracle's single
  precision build states how far float arithmetic alone drifts.

About five minutes on two cores:
    python tests/golden/make_large_1024.py
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

STEPS = 3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_1024.txt")
SAMPLE_SEED = 1024
N_SAMPLE = 4096


def run(prec, gamma, path):
    P = synth.config_problem("large_1024", with_truth=False)
    g = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    t0 = time.time()
    x, t, _ = ora.eg(g, P.mu, P.I, P.y.astype(np.float64), np.zeros(P.d), gamma, STEPS, prec=prec)
    np.save(path, x)
    print("%s: %d steps in %.0f s" % (prec, t, time.time() - t0), flush=True)


def main():
    P = synth.config_problem("large_1024", with_truth=True)
    g = ora.Geom(P.n_pix, P.n_views, P.n_bins)
    y64 = P.y.astype(np.float64)
    t0 = time.time()
    rows = ora.forward(g, np.ones(g.d))
    cols = ora.back(g, np.ones(g.n))
    lam = rows.max() * cols.max() / g.n
    gamma = ora.step_size(lam, P.mu, P.I)
    print("lambda bound %.12e (%.0f s); gamma %.12e" % (lam, time.time() - t0, gamma), flush=True)
    tmp = {p: OUT + "." + p + ".npy" for p in ("f64", "f32")}
    procs = [Process(target=run, args=(p, gamma, tmp[p])) for p in ("f64", "f32")]
    for p in procs:
        p.start()
    # the operator at 0.9 x_true meanwhile
    x = (0.9 * P.x_true).astype(np.float32).astype(np.float64)
    F, s, r = ora.operator(g, P.mu, P.I, y64, x, want_sr=True)
    _, m = ora.residual(s, P.mu, P.I, y64)
    Y = y64.reshape(P.Wn, -1).sum(0)
    rng = np.random.default_rng(SAMPLE_SEED)
    pix = np.sort(rng.choice(P.d, size=N_SAMPLE, replace=False))
    rays = np.sort(rng.choice(g.n, size=N_SAMPLE, replace=False))
    fscale = ora.back_pixels(g, Y + m, pix) / g.n
    for p in procs:
        p.join()
    x64, x32 = np.load(tmp["f64"]), np.load(tmp["f32"])
    lines = ["# EXACT oracle on workload large_1024 (written by tests/golden/make_large_1024.py,",
             "# oracle only).  y checksum = sum of all counts; samples drawn with seed %d."
             % SAMPLE_SEED,
             "steps = %d" % STEPS,
             "lambda_bound = %.17g" % lam,
             "gamma = %.17g" % gamma,
             "y_sum = %.17g" % float(y64.sum()),
             "x_norm = %.17g" % float(np.linalg.norm(x64)),
             "f32_rel_l2 = %.6e" % (np.linalg.norm(x32 - x64) / np.linalg.norm(x64)),
             "# F at x = float32(0.9 x_true): pixel F scale",
             "[F]"]
    lines += ["%d %.17g %.17g" % (p, F[p], fscale[k]) for k, p in enumerate(pix)]
    lines += ["# r at the same x: ray r scale", "[r]"]
    lines += ["%d %.17g %.17g" % (i, r[i], Y[i] + m[i]) for i in rays]
    lines += ["# iterate after the steps: pixel value", "[x]"]
    lines += ["%d %.17g" % (p, x64[p]) for p in pix]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    for p in tmp.values():
        if os.path.exists(p):
            os.remove(p)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
