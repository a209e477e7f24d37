"""Build-time autotuner for the projector kernels' tile knobs.

    python -m paper_2503_19925_amd.tune build          # compile every variant (no GPU needed)
    python -m paper_2503_19925_amd.tune time           # time them on the GPU, write tuned.json
    python -m paper_2503_19925_amd.build               # rebuild libexact.so with the choice

Knobs (compile-time macros of exact_kernels.hip):
  EXACT_LINE_BATCH  image lines per software-pipelined batch of the forward
                    projector (the next batch's loads are in flight while a
                    batch is summed)
  EXACT_VIEW_BATCH  views per batch of the back-projector, likewise
  EXACT_FWD_SEGS    waves per forward workgroup (each takes a share of the
                    lines of the workgroup's 128 rays, two per lane)

One choice serves every shape.  Each knob changes the order of the float
sums, and a batched run must reproduce its solo run bit for bit, so all
runs of one build share one arithmetic order.

Objective: the geometric mean of extragradient steps per second over three
shape classes (256^2 x 180 views x 363 bins, 512^2 x 180 x 725, 1024^2 x
720 x 1448), each a resident solver timed with HIP events over graph
replays, best of three repeats per pass and of two passes over all
variants.  A variant replaces the sources' defaults only if it beats them
by more than 1 % (about the run-to-run spread).

Correctness gate: every variant also runs a short solve (40 steps of the
256^2 class from x = 0 with Theorem 2's step size); a variant whose iterate
differs from the default build's by more than 1e-5 relative L2, or whose
last residual rho differs by more than 1e-4 relative, is rejected (its sums
run in another order, so bitwise equality is not expected, but a wrong
reduction or a broken kernel shows far above these bounds).
"""
import itertools
import json
import math
import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from paper_2503_19925_amd import build as libbuild  # noqa: E402

VARIANT_DIR = os.path.join(HERE, "_tune")
GRID = {"EXACT_LINE_BATCH": (2, 4, 6, 8), "EXACT_VIEW_BATCH": (2, 4, 6), "EXACT_FWD_SEGS": (2, 4, 8)}
DEFAULT = dict(libbuild.DEFAULT_KNOBS)
# (name, N, V, B, K, Wn, I0, timed steps)
CLASSES = [("256", 256, 180, 363, 30, 3, 1e4, 400), ("512", 512, 180, 725, 30, 3, 1e4, 300),
           ("1024", 1024, 720, 1448, 64, 4, 1e3, 60)]
MARGIN = 1.01
GATE_STEPS, GATE_GAMMA = 40, 0.0    # gamma 0: Theorem 2's rule by power iteration


def variants():
    keys = sorted(GRID)
    for vals in itertools.product(*(GRID[k] for k in keys)):
        yield dict(zip(keys, vals))


def tag(knobs):
    return "L%d_V%d_S%d" % (knobs["EXACT_LINE_BATCH"], knobs["EXACT_VIEW_BATCH"],
                            knobs["EXACT_FWD_SEGS"])


def lib_path(knobs):
    return os.path.join(VARIANT_DIR, "lib_%s.so" % tag(knobs))


def cmd_build(jobs=6):
    os.makedirs(VARIANT_DIR, exist_ok=True)
    todo = list(variants())
    t0 = time.time()

    def one(k):
        libbuild.build(out=lib_path(k), knobs=k)
        return tag(k)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for name in ex.map(one, todo):
            print("built", name, "(%.0f s)" % (time.time() - t0), flush=True)


def time_one(path):
    """Runs in a child process: ms per EG step of each shape class with the
    library at `path`."""
    import torch
    from paper_2503_19925_amd import exact, synth
    exact.LIB_PATH = path
    exact.load()
    out = {}
    for name, N, V, B, K, Wn, I0, steps in CLASSES:
        P = synth.make_problem("tune" + name, N, V, B, K, Wn, I0, 20, 7000 + N, 8000 + N,
                               with_truth=False)
        g = exact.Geometry(N, V, B)
        y = torch.as_tensor(P.y, device="cuda")
        x = torch.zeros(g.d, device="cuda")
        sv = exact.Solver(g, P.mu, P.I, y, x, max_iters=1 << 30)
        sv.step(10)
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sv.step(steps)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        sv.close()
        g.close()
        out[name] = best
    # the correctness gate's short solve
    name, N, V, B, K, Wn, I0, _ = CLASSES[0]
    P = synth.make_problem("tune" + name, N, V, B, K, Wn, I0, 20, 7000 + N, 8000 + N,
                           with_truth=False)
    g = exact.Geometry(N, V, B)
    x = torch.zeros(g.d, device="cuda")
    info = exact.exact_solve(g, P.mu, P.I, torch.as_tensor(P.y, device="cuda"), x,
                             gamma=GATE_GAMMA, max_iters=GATE_STEPS)
    gate = {"x": x.cpu().numpy().astype("float64").tolist(), "rho": info["resid"]}
    g.close()
    prop = torch.cuda.get_device_properties(0)
    dev = "%s (%s)" % (prop.name, getattr(prop, "gcnArchName", "?"))
    print(json.dumps({"ms": out, "device": dev, "gate": gate}), flush=True)


def cmd_time(report=None, passes=2, per_run_timeout=300):
    rows = {tag(k): dict(knobs=k, ms={}) for k in variants()}
    missing = [t for t, r in rows.items() if not os.path.exists(lib_path(r["knobs"]))]
    if missing:
        raise SystemExit("variants not built: %s (run `tune build`)" % ", ".join(missing))
    device = None
    for p in range(passes):
        for t, r in rows.items():
            print("[tune] pass %d variant %s" % (p + 1, t), flush=True)
            res = subprocess.run([sys.executable, "-m", "paper_2503_19925_amd.tune", "_one",
                                  lib_path(r["knobs"])], cwd=ROOT, capture_output=True,
                                 text=True, timeout=per_run_timeout)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise SystemExit("timing run of %s failed (exit %d)" % (t, res.returncode))
            rec = json.loads(res.stdout.strip().splitlines()[-1])
            device = rec["device"]
            r["gate"] = rec["gate"]
            for c, ms in rec["ms"].items():
                r["ms"][c] = min(r["ms"].get(c, math.inf), ms)
            print("[tune]   %s" % " ".join("%s:%.4f" % kv for kv in sorted(rec["ms"].items())),
                  flush=True)
    base = rows[tag(DEFAULT)]
    xb, rb = base["gate"]["x"], base["gate"]["rho"]
    nb = math.sqrt(sum(v * v for v in xb))
    for t, r in rows.items():
        r["score"] = math.exp(sum(math.log(1e3 / ms) for ms in r["ms"].values()) / len(r["ms"]))
        dx = math.sqrt(sum((a - b) ** 2 for a, b in zip(r["gate"]["x"], xb))) / nb
        drho = abs(r["gate"]["rho"] - rb) / abs(rb)
        r["gate_ok"] = dx <= 1e-5 and drho <= 1e-4
        if not r["gate_ok"]:
            print("[tune] %s rejected: iterate differs by %.2e, rho by %.2e" % (t, dx, drho),
                  flush=True)
            r["score"] = 0.0
        del r["gate"]
    best = max(rows.values(), key=lambda r: r["score"])
    chosen = best if best["score"] > MARGIN * base["score"] else base
    rec = {"knobs": chosen["knobs"], "score_steps_per_s": chosen["score"],
           "default_score_steps_per_s": base["score"], "best": tag(best["knobs"]),
           "margin": MARGIN, "device": device, "classes": [c[:4] for c in CLASSES],
           "table": sorted(([tag(r["knobs"]), r["ms"], r["score"]] for r in rows.values()),
                           key=lambda x: -x[2])}
    with open(libbuild.TUNED, "w") as f:
        json.dump(rec, f, indent=1)
    print("[tune] chosen %s (score %.1f steps/s; default %.1f; best %s)"
          % (tag(chosen["knobs"]), chosen["score"], base["score"], tag(best["knobs"])), flush=True)
    if report:
        write_report(rec, report)


def write_report(rec, path):
    lines = ["# Tile-knob sweep (autotuner)", "",
             "Every combination of the forward's line batch (L), the back-projector's view",
             "batch (V) and the forward's waves per workgroup (S), timed as resident",
             "solvers on three shape classes (ms per EG step, best of 3 repeats x 2",
             "passes). Score: geometric mean of steps/s over the classes. Device: %s." %
             rec["device"], "",
             "Command (from the repository root):", "", "```",
             "python -m paper_2503_19925_amd.tune build && "
             "python -m paper_2503_19925_amd.tune time --report profiles/tuning_sweep.md",
             "```", "",
             "Chosen: **%s** (score %.1f steps/s; the sources' defaults L4_V4_S4 score %.1f;"
             " a variant must beat them by %d %% to replace them)." %
             (tag(rec["knobs"]), rec["score_steps_per_s"], rec["default_score_steps_per_s"],
              round((rec["margin"] - 1) * 100)), "",
             "| variant | 256² ×180 | 512² ×180 | 1024² ×720 | score (steps/s) |",
             "|---|---|---|---|---|"]
    for t, ms, score in rec["table"]:
        lines.append("| %s | %.4f | %.4f | %.4f | %.1f |" % (t, ms["256"], ms["512"], ms["1024"],
                                                           score))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    a = sys.argv[1:]
    if a[:1] == ["build"]:
        cmd_build()
    elif a[:1] == ["time"]:
        cmd_time(report=a[a.index("--report") + 1] if "--report" in a else None)
    elif a[:1] == ["_one"]:
        time_one(a[1])
    else:
        raise SystemExit(__doc__)
