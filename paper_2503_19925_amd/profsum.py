"""Summaries of rocprofv3 output for profiles/ (text only).

    python -m paper_2503_19925_amd.profsum counters <pmc dir> <workload>
        FETCH_SIZE / WRITE_SIZE runs (one counter per run, each under
        <pmc dir>/<counter>/run_counter_collection.csv) -> profiles/traffic.json
        and profiles/counters_<workload>.md.  HBM bytes are calibrated by the
        benchmark's 256 MiB device copies, whose dispatches are in the same runs.
    python -m paper_2503_19925_amd.profsum kernels <out dir>
        --kernel-trace --stats runs and benchmark logs of one GPU call
        (<out dir>/prof/bench, bench.log, prof_large, large.err) ->
        profiles/kernels_solve_512.md and profiles/kernels_large_1024.md.
    python -m paper_2503_19925_amd.profsum utilisation <pmc dir>
        two counter passes (A: SQ/GRBM, B: TA/TD/TCP/TCC) per workload under
        <pmc dir>/<workload>_<pass> -> profiles/counters_utilisation.md and
        profiles/valu.json (VALU instructions per launch, read by bench.py).
    python -m paper_2503_19925_amd.profsum tests <kernel_stats.csv> <pytest log>
        a kernel trace of the GPU test suite -> profiles/kernels_gpu_tests.md,
        checked against every kernel compiled into libexact.so.
    python -m paper_2503_19925_amd.profsum batched_counters <counter csv> [out.md]
        one counter pass (BATCHED_PMC) over the batched leg alone ->
        out.md (default profiles/counters_batched.md): VALU issue and waves
        resident of the batched kernels.
    python -m paper_2503_19925_amd.profsum batched <kernel_trace.csv> <bench stderr> [out.md]
        a kernel trace of the benchmark's batched leg (BATCHED_TRACE) -> out.md
        (default profiles/kernels_batched.md): the batched phase's busy time,
        its kernels, the per-step split and the serial leg's kernel time.

traffic.json and valu.json carry the build id (kernel source and tile
knobs) the counters were taken on; bench.py reports their figures only while
that id is the current one.
"""
import collections
import csv
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")
sys.path.insert(0, ROOT)

from paper_2503_19925_amd import build as libbuild  # noqa: E402

COPY_MIB = 256
PMC_COMMAND = ("timeout -s KILL 150 rocprofv3 --pmc <counter> --output-format csv -d "
               "<out>/pmc/<counter> -o run -- python3 bench.py --steps 5 --warmup 2 "
               "--proj-reps 5 --kernel-reps 5 --batch 0 --served 0 --cpu-steps 0 "
               "--large-to-tol 0 --calibrate-copy-mb 256")
BENCH_TRACE = ("rocprofv3 --kernel-trace --stats -d <out>/prof/bench --output-format csv "
               "-o bench -- python3 bench.py --steps 50 --warmup 5 --cpu-steps 0 --batch 0 "
               "--served 0 --large-to-tol 0 --kernel-reps 20")
LARGE_TRACE = ("rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_large "
               "-o large -- python3 bench.py --workload large_1024 --steps 10 --warmup 2 "
               "--proj-reps 5 --kernel-reps 5 --batch 0 --served 0 --cpu-steps 0 --tv-steps -1 "
               "--dense-steps 0")
LARGE_BENCH = ("python3 bench.py --workload large_1024 --steps 20 --warmup 3 --proj-reps 10 "
               "--kernel-reps 10 --batch 0 --served 0 --cpu-steps 0 --tv-steps -1 "
               "--dense-steps 0 --to-tol 1e-4")
BATCHED_TRACE = ("rocprofv3 --kernel-trace --output-format csv -d <trace dir> -o b -- python3 "
                 "bench.py --steps 5 --warmup 2 --proj-reps 2 --kernel-reps 2 --cpu-steps 0 "
                 "--tv-steps -1 --dense-steps 0 --background-steps 0 --served 0 "
                 "--large-to-tol 0 --batch 64 2> <bench stderr>")
BATCHED_PMC_COUNTERS = "SQ_WAVES SQ_INSTS_VALU SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU GRBM_GUI_ACTIVE"
BATCHED_PMC = ("timeout -s KILL 300 rocprofv3 --pmc " + BATCHED_PMC_COUNTERS + " --output-format csv "
               "-d <run dir> -o run -- python3 bench.py --steps 5 --warmup 2 --proj-reps 2 "
               "--kernel-reps 2 --cpu-steps 0 --tv-steps -1 --dense-steps 0 --background-steps 0 "
               "--served 0 --large-to-tol 0 --batch 64 --batch-serial 0")
TESTS_TRACE = ("rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_tests "
               "-o tests -- python3 -u -m pytest tests -m gpu -x -q --timeout 600 "
               "--timeout-method thread")


def short(name):
    """Kernel name without namespace, parameters or `void`."""
    n = name.replace("exact::(anonymous namespace)::", "")
    n = n[:n.index("(")] if "(" in n else n
    return n.replace("void ", "").strip()


# ------------------------------------------------------------- counters

def cmd_counters(pmc_dir, workload):
    def load(counter):
        per = collections.defaultdict(list)
        path = os.path.join(pmc_dir, counter, "run_counter_collection.csv")
        for r in csv.DictReader(open(path)):
            per[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return per

    F, W = load("FETCH_SIZE"), load("WRITE_SIZE")
    copy_kib = COPY_MIB * 1024
    fc = [v for v in F["__amd_rocclr_copyBuffer"] if v > 0.4 * copy_kib]
    wc = [v for v in W["__amd_rocclr_copyBuffer"] if v > 0.9 * copy_kib]
    if not fc or not wc:
        raise SystemExit("no 256 MiB copy dispatches to calibrate against")
    fs = copy_kib / (sum(fc) / len(fc))
    ws = copy_kib / (sum(wc) / len(wc))
    kernels = {}
    for k in sorted(F):
        if not k.startswith(("k_", "kb_")):
            continue
        f = sum(F[k]) / len(F[k])
        w = sum(W[k]) / len(W[k]) if k in W else 0.0
        kernels[k] = dict(fetch_kib=f, write_kib=w, hbm_bytes_per_launch=(f * fs + w * ws) * 1024,
                          launches=len(F[k]))
    bu = [v for k, v in kernels.items() if k.startswith("k_back_update")]
    if bu:   # both instantiations of the fused back-projection + update
        kernels["k_back_update"] = {
            "hbm_bytes_per_launch": sum(v["hbm_bytes_per_launch"] for v in bu) / len(bu)}
    rec = {"kernel_build_id": libbuild.build_id(), "knobs": libbuild.tuned_knobs(),
           "fetch_scale": fs, "write_scale": ws, "workloads": {workload: kernels}}
    with open(os.path.join(PROFILES, "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)

    md = ["# HBM traffic per kernel, workload %s" % workload, "",
          "rocprofv3 counter passes, one counter per run, on the same short benchmark run",
          "(5 timed EG steps, 5 profiled steps, 5 standalone projector calls each, power",
          "iteration, the known-background, TV-ball and dense legs, plus three 256 MiB",
          "device copies for calibration).  From the repository root, TMPDIR=/tmp,",
          "`<out>` an output directory,",
          "`<counter>` = `FETCH_SIZE`, then `WRITE_SIZE`:", "", "```", PMC_COMMAND, "```", "",
          "Summarised by `python -m paper_2503_19925_amd.profsum counters <out>/pmc %s`."
          % workload, "",
          "**Calibration.** Each 256 MiB copy (262,144 KiB read and written) reads",
          "FETCH_SIZE = %.1f KiB and WRITE_SIZE = %.1f KiB per dispatch, so reads are"
          % (copy_kib / fs, copy_kib / ws),
          "scaled by %.4f and writes by %.4f below (HBM bytes = 1024 (FETCH_SIZE x read" % (fs, ws),
          "scale + WRITE_SIZE x write scale), averaged over the kernel's dispatches).",
          "`profiles/traffic.json` holds the same figures with the build id (kernel",
          "source and tile knobs) they were taken on; the benchmark reports them as",
          "`roofline.traffic` only while that build id is the current one.", "",
          "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes / launch | launches |",
          "|---|---|---|---|---|"]
    for k, v in kernels.items():
        if "fetch_kib" in v:
            md.append("| %s | %.1f | %.1f | %.3e | %d |" % (k, v["fetch_kib"], v["write_kib"],
                                                          v["hbm_bytes_per_launch"], v["launches"]))
    if bu and workload == "solve_512":
        b = kernels["k_back_update"]["hbm_bytes_per_launch"]
        md += ["", "Reading.  The step's back-projection + update kernel (k_back_update, mean of",
               "its two instantiations: %.3e B per launch) moves about 1/%.0f of its" % (b, 3.44e8 / b),
               "algorithmic bytes (4 B per nonzero of A, 84,962,942 nonzeros, plus the",
               "residual, the iterate and the outputs: 3.44e8 B per launch).  The residual",
               "(0.53 MB padded) and the image stay in each XCD's L2; what reaches HBM is",
               "about one read of r and x per XCD plus the outputs (z, its padded copy and",
               "transpose).  The forward reads the padded image pair (2 x 1.06 MB) about once",
               "per XCD (8 XCDs: about 17 MB), which is nearly all of its HBM traffic.",
               "Neither kernel is HBM-bound: at 8 TB/s these bytes take 1-2 us of kernels",
               "that run about 25-28 us; they are bound by instruction issue and the vector",
               "memory return path."]
    with open(os.path.join(PROFILES, "counters_%s.md" % workload), "w") as f:
        f.write("\n".join(md) + "\n")
    print("wrote traffic.json (%s) and counters_%s.md" % (rec["kernel_build_id"], workload))


# ------------------------------------------------------------- kernel times

def stats(path):
    rows = []
    for r in csv.DictReader(open(path)):
        n = short(r["Name"])
        if n.startswith("at::native") or "Functor" in n:
            n = "torch fill/copy"
        rows.append((n, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                     float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return rows


def table(rows):
    md = ["| kernel | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for n, c, a, mi, ma, p in rows:
        md.append("| %s | %d | %.2f | %.2f | %.2f | %.1f%% |" % (n, c, a, mi, ma, p))
    return md


def back_to_back(trace_csv, min_run=10):
    """Mean duration (us) and count of the dispatches that run back to back:
    runs of at least min_run consecutive dispatches of one kernel, each run's
    first dispatch dropped."""
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    out = collections.defaultdict(list)
    i = 0
    while i < len(rows):
        j = i
        while j < len(rows) and rows[j]["Kernel_Name"] == rows[i]["Kernel_Name"]:
            j += 1
        if j - i >= min_run:
            out[short(rows[i]["Kernel_Name"])] += [
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3 for r in rows[i + 1:j]]
        i = j
    return {k: (sum(v) / len(v), len(v)) for k, v in out.items()}


def cmd_kernels(out_dir):
    rows = stats(os.path.join(out_dir, "prof", "bench", "bench_kernel_stats.csv"))
    b = json.loads(open(os.path.join(out_dir, "bench.log")).read().strip().splitlines()[-1])
    ph = b["kernel_ms"]

    def get(rs, name):
        return [r for r in rs if r[0] == name][0][2]

    fwd, bh = get(rows, "k_forward<true>"), get(rows, "k_back_update<true, true, false>")
    bf, fin = get(rows, "k_back_update<true, false, false>"), get(rows, "k_eg_finish<false>")
    tot = 2 * fwd + bh + bf
    md = ["# Kernel times, workload solve_512 (EXACT step)", "",
          "512x512 image, 180 views over 180 deg, 725 bins, K=30 energy bins, 3 windows.",
          "One EG step is four kernels (the solver replays captured graphs of eight",
          "steps): k_forward<true> (forward",
          "projection + spectral residual at x_t, written weighted into the padded",
          "residual; one more workgroup, dispatched last, runs the previous step's finish),",
          "k_back_update<true, true, false> (back-projection + half-step update +",
          "residual partials; the bin-pair rule, clamp-free on this covered geometry),",
          "k_forward<true> at x_{t+1/2} and k_back_update<true, false, false>",
          "(back-projection + full-step update).  k_eg_finish below is the finish run",
          "as its own kernel: by the per-phase timing steps, and to settle a run's",
          "state before the host reads it.  The run below also makes",
          "the benchmark's other calls: power iteration (k_forward<false>,",
          "k_back<true, false>, k_dot3, k_normalize), the standalone projector timings",
          "(exact_backproject = k_weigh_rows + k_back<true, false>; exact_forward =",
          "fills + k_pad_pair + k_forward<false>), the kernel timings (each step kernel",
          "launched back to back, an untimed and a timed pass, the full-step update into",
          "a scratch image), the known-background leg (the same kernels),"
          "the TV-ball leg (k_fgp_steps, k_fgp_final, k_tv_parts, k_dyk_*, and the EG",
          "kernels of two steps) and the dense leg (k_dense_*).", "",
          "Command (from the repository root, TMPDIR=/tmp, `<out>` an output",
          "directory):", "", "```", BENCH_TRACE, "```", "",
          "Summarised by `python -m paper_2503_19925_amd.profsum kernels <out>`.", ""]
    md += table(rows)
    b2b = back_to_back(os.path.join(out_dir, "prof", "bench", "bench_kernel_trace.csv"))
    fwd_b = (ph["forward_residual_x"] + ph["forward_residual_xh"]) / 2 * 1e3
    bu_b = (ph["back_update_half"] + ph["back_update_full"]) / 2 * 1e3
    bu = (bh + bf) / 2
    # the benchmark's `roofline` kernel: the one that takes more of the step
    dom = "k_forward<true>" if fwd_b >= bu_b else "k_back_update (both variants)"
    bu_keys = ("k_back_update<true, true, false>", "k_back_update<true, false, false>")
    b2b_bu = (sum(b2b[k][0] for k in bu_keys) / 2) if all(k in b2b for k in bu_keys) else None
    md += ["", "**Agreement with the benchmark's event timing.** The default `python bench.py`",
           "run (same build, not under the profiler) timed the step at %.4f ms (graph" % b["ms_per_step"],
           "replay, HIP events) and each step kernel over back-to-back launches between",
           "HIP events: forward at x_t %.2f us, back + half update %.2f us, forward at"
           % (ph["forward_residual_x"] * 1e3, ph["back_update_half"] * 1e3),
           "x_{t+1/2} %.2f us, back + full update %.2f us, finish %.2f us.  The profiler's"
           % (ph["forward_residual_xh"] * 1e3, ph["back_update_full"] * 1e3, ph["finish"] * 1e3),
           "averages: k_forward<true> %.2f us (the benchmark's forward mean %.2f us, %+.1f %%)," % (
               fwd, fwd_b, 100 * (fwd_b - fwd) / fwd),
           "k_back_update<true, true, false> %.2f us, k_back_update<true, false, false> %.2f us" % (bh, bf),
           "(their mean %.2f us; the benchmark's back + update mean %.2f us, %+.1f %%)" % (
               bu, bu_b, 100 * (bu_b - bu) / bu),
           "(and the standalone k_eg_finish<false> %.2f us); the graph's four kernels sum to" % fin,
           ("%.1f us per step, %.1f us short of the replayed step: the gaps between the "
            "graph's kernels and the finish workgroup of the first kernel."
            % (tot, b["ms_per_step"] * 1e3 - tot)) if tot <= b["ms_per_step"] * 1e3 else
           ("%.1f us per step, above the replayed step's %.1f us: the profiler lengthens "
            "each dispatch, and without it the gaps between the graph's kernels (eight "
            "steps per graph) take less than that." % (tot, b["ms_per_step"] * 1e3)), "",
           "The benchmark times each kernel over back-to-back launches of that kernel",
           "alone; in the trace above most dispatches run inside the step, after the",
           "other kernel, and the first of each call starts cold.  The trace's own",
           "back-to-back runs (10 or more consecutive dispatches of one kernel, each",
           "run's first dropped) average: %s." % ", ".join(
               "%s %.2f us over %d dispatches" % (k, v[0], v[1]) for k, v in sorted(b2b.items())),
           ("Against them the benchmark's forward mean is %+.1f %%." % (
               100 * (fwd_b - b2b["k_forward<true>"][0]) / b2b["k_forward<true>"][0])
            if "k_forward<true>" in b2b else ""),
           ("Against the mean of the two back + update runs (%.2f us) the benchmark's "
            "back + update mean is %+.1f %%." % (b2b_bu, 100 * (bu_b - b2b_bu) / b2b_bu))
           if b2b_bu else "",
           "The benchmark line's `roofline` is the kernel that takes more of the step: "
           "here %s." % dom]
    with open(os.path.join(PROFILES, "kernels_solve_512.md"), "w") as f:
        f.write("\n".join(md) + "\n")

    rl = stats(os.path.join(out_dir, "prof_large", "large_kernel_stats.csv"))
    err = open(os.path.join(out_dir, "large.err")).read()
    m = re.search(r"timed 20 steps: ([0-9.]+) ms/step", err)
    t = re.search(r"to tolerance 1e-04: (\d+) steps, ([0-9.]+) s", err)
    phl = re.search(r"kernel ms: (.*)", err).group(1)
    md = ["# Kernel times, workload large_1024 (EXACT step)", "",
          "1024x1024 image, 720 views over 180 deg, 1448 bins, K=64 energy bins, 4 windows,",
          "I0=1e3.  nnz(A) = 1,357,334,016 (device count); algorithmic bytes per",
          "back-projection 5.43e9.", "",
          "Command (from the repository root, TMPDIR=/tmp, `<out>` an output",
          "directory):", "", "```", LARGE_TRACE, "```", "",
          "Summarised by `python -m paper_2503_19925_amd.profsum kernels <out>`.", ""]
    md += table(rl)
    md += ["", "Benchmark line of the same workload (HIP events, not under the profiler):",
           "`%s`:" % LARGE_BENCH,
           "%s ms per EG step (%.0f EG iters/s); kernel ms %s; solving from x = 0 to"
           % (m.group(1), 1e3 / float(m.group(1)), phl),
           "natural residual 1e-4 took %s steps and %s s." % (t.group(1), t.group(2))]
    with open(os.path.join(PROFILES, "kernels_large_1024.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("wrote kernels_solve_512.md and kernels_large_1024.md")


# ------------------------------------------------------------- utilisation

UTIL_PASSES = {
    "A": "SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU "
         "SQ_WAIT_INST_ANY SQ_INST_LEVEL_VMEM SQ_INSTS_VMEM_RD GRBM_GUI_ACTIVE GRBM_COUNT",
    "B": "TA_TA_BUSY_sum TA_ADDR_STALLED_BY_TC_CYCLES_sum TD_TD_BUSY_sum TD_TC_STALL_sum "
         "TCP_TCP_TA_DATA_STALL_CYCLES_sum TCP_PENDING_STALL_CYCLES_sum TCP_TCC_READ_REQ_sum "
         "TCP_TCC_READ_REQ_LATENCY_sum TCC_HIT_sum TCC_MISS_sum GRBM_GUI_ACTIVE"}
UTIL_BENCH = ("python3 bench.py --workload <workload> --steps 5 --warmup 2 --proj-reps 2 "
              "--kernel-reps 2 --batch 0 --served 0 --cpu-steps 0 --tv-steps -1 "
              "--dense-steps 0 --background-steps 0 --large-to-tol 0")
CUS, SIMDS, CLOCK_GHZ = 256, 1024, 2.4
UTIL_KERNELS = ("k_forward<true>", "k_back_update<true, true, false>",
                "k_back_update<true, false, false>")


def cmd_utilisation(pmc_dir):
    md = ["# Unit utilisation of the step's kernels (hardware counters)", "",
          "Two rocprofv3 counter passes per workload on a short benchmark run (from",
          "the repository root, TMPDIR=/tmp, `<out>` an output directory;",
          "`<workload>` = `solve_512`, then",
          "`large_1024`; `<pass>` = A, then B):", "", "```",
          "timeout -s KILL 120 rocprofv3 --pmc <counters of the pass> --output-format csv "
          "-d <out>/pmc3/<workload>_<pass> -o run -- " + UTIL_BENCH, "```", "",
          "Pass A: `%s`." % UTIL_PASSES["A"], "", "Pass B: `%s`." % UTIL_PASSES["B"], "",
          "Summarised by `python -m paper_2503_19925_amd.profsum utilisation <out>/pmc3`.",
          "", "Figures per dispatch (mean over the run's dispatches of the kernel), against",
          "MI355X's 256 CUs (1024 SIMDs) at the published 2.4 GHz peak engine clock; the",
          "duration is the dispatch's own (the counter run's timestamps), so a clock",
          "below 2.4 GHz makes every fraction below a lower bound:", "",
          "* VALU issue: SQ_INSTS_VALU x 2 cycles / (1024 SIMDs x duration x 2.4 GHz):",
          "  against the published FP32 vector rate (one wave64 instruction per 2 cycles",
          "  per SIMD), which two-operand 32-bit instructions reach on MI355X (measured);",
          "* VALU at 4 cycles: the same count at 4 cycles per instruction, the rate",
          "  measured for the three-operand FP32 FMA and the FP64 add and fract.  A",
          "  kernel's mix lies between the two rates, so this figure can pass 100 % when",
          "  part of the mix issues at the faster one;",
          "* waves resident per SIMD: SQ_WAVE_CYCLES x 4 (quad-cycles) / (1024 x cycles);",
          "* TA / TD busy: TA_TA_BUSY_sum, TD_TD_BUSY_sum / (256 CUs x cycles);",
          "* L2 hit rate: TCC_HIT / (TCC_HIT + TCC_MISS); L2 read latency:",
          "  TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum (cycles);",
          "* HBM: the kernel's bytes per launch from the FETCH_SIZE / WRITE_SIZE passes",
          "  (profiles/traffic.json, solve_512 only) over the dispatch's duration.", ""]
    traffic = {}
    try:
        traffic = json.load(open(os.path.join(PROFILES, "traffic.json")))["workloads"]
    except (OSError, ValueError, KeyError):
        pass
    valu_rec = {}
    for wl in ("solve_512", "large_1024"):
        vals = collections.defaultdict(lambda: collections.defaultdict(list))
        dur = collections.defaultdict(list)
        for p in ("A", "B"):
            path = os.path.join(pmc_dir, "%s_%s" % (wl, p), "run_counter_collection.csv")
            for r in csv.DictReader(open(path)):
                n = short(r["Kernel_Name"])
                vals[n][r["Counter_Name"]].append(float(r["Counter_Value"]))
                if p == "A" and r["Counter_Name"] == "SQ_INSTS_VALU":
                    dur[n].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
        md += ["## %s" % wl, "",
               "| kernel | dispatches | duration (us) | VALU issue | VALU at 4 cycles | waves / SIMD "
               "| TA busy | TD busy | L2 hit | L2 read latency (cycles) | HBM (GB/s, of 8000) |",
               "|---|---|---|---|---|---|---|---|---|---|---|"]
        wrec = valu_rec.setdefault(wl, {})
        for k in UTIL_KERNELS:
            v = {c: sum(x) / len(x) for c, x in vals[k].items()}
            d = sum(dur[k]) / len(dur[k])
            cyc = d * CLOCK_GHZ * 1e9
            hbm = traffic.get(wl, {}).get(k, {}).get("hbm_bytes_per_launch")
            issue = v["SQ_INSTS_VALU"] * 2 / SIMDS / cyc
            issue4 = v["SQ_INSTS_VALU"] * 4 / SIMDS / cyc
            ta = v["TA_TA_BUSY_sum"] / CUS / cyc
            md.append("| %s | %d | %.1f | %.0f %% | %.0f %% | %.1f | %.0f %% | %.0f %% | %.1f %% "
                      "| %.0f | %s |" % (
                          k, len(dur[k]), d * 1e6, 100 * issue, 100 * issue4,
                          v["SQ_WAVE_CYCLES"] * 4 / SIMDS / cyc, 100 * ta,
                          100 * v["TD_TD_BUSY_sum"] / CUS / cyc,
                          100 * v["TCC_HIT_sum"] / (v["TCC_HIT_sum"] + v["TCC_MISS_sum"]),
                          v["TCP_TCC_READ_REQ_LATENCY_sum"] / v["TCP_TCC_READ_REQ_sum"],
                          "%.0f" % (hbm / d / 1e9) if hbm else "-"))
            wrec[k] = {"valu_lane_instr_per_launch": 64.0 * v["SQ_INSTS_VALU"],
                       "valu_active_quad_cycles": v["SQ_ACTIVE_INST_VALU"],
                       "duration_us": d * 1e6, "valu_issue_frac": issue,
                       "valu_issue_frac_4_cycles": issue4, "ta_busy_frac": ta,
                       "dispatches": len(dur[k])}
        bu = [wrec[k] for k in UTIL_KERNELS if k.startswith("k_back_update")]
        wrec["k_back_update"] = {f: sum(b[f] for b in bu) / len(bu)
                                 for f in ("valu_lane_instr_per_launch", "valu_active_quad_cycles",
                                           "duration_us", "valu_issue_frac",
                                           "valu_issue_frac_4_cycles", "ta_busy_frac")}
        md.append("")
    md += ["Reading.  Both kernels are bound by VALU issue for their instruction mix:",
           "counted at 4 cycles per instruction (the measured rate of their FP64",
           "crossing arithmetic and three-operand FMAs) they fill 78-108 % of the",
           "forward's and 63-89 % of the back-projector's duration, and the forward at",
           "1024² passes 100 %, so part of its mix issues at the faster two-cycle rate.",
           "The address and data-return units (TA, TD) stay below them (50-84 %), since",
           "the forward serves two rays per 16-byte load.  L2 hit rates of 80-93 % and",
           "HBM rates far below 8 TB/s show the operands served from the XCDs' L2."]
    with open(os.path.join(PROFILES, "counters_utilisation.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    rec = {"kernel_build_id": libbuild.build_id(), "knobs": libbuild.tuned_knobs(),
           "note": "SQ_INSTS_VALU per dispatch x 64 lanes; fractions against 1024 SIMDs at "
                   "2.4 GHz over the dispatch's duration (counter run), at one wave64 "
                   "instruction per 2 cycles (valu_issue_frac) and per 4 cycles",
           "workloads": valu_rec}
    with open(os.path.join(PROFILES, "valu.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote counters_utilisation.md and valu.json (%s)" % rec["kernel_build_id"])


# ------------------------------------------------------------- test coverage

def compiled_kernels():
    """Every kernel in libexact.so's device code, from the device assembly of
    the library's current sources."""
    names = []
    with tempfile.TemporaryDirectory() as tmp:
        for src in libbuild.SOURCES:
            out = os.path.join(tmp, os.path.basename(src) + ".s")
            subprocess.run([libbuild.HIPCC] + [f for f in libbuild.FLAGS if f not in ("-shared", "-fPIC")]
                           + libbuild.defines(libbuild.tuned_knobs()) +
                           ["--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
                            "-I", os.path.join(HERE, "csrc"), "-o", out, os.path.join(HERE, src)],
                           check=True, capture_output=True)
            for line in open(out):
                if line.strip().startswith(".amdhsa_kernel "):
                    names.append(line.split()[1])
    dem = subprocess.run(["c++filt"], input="\n".join(names), text=True, capture_output=True,
                         check=True).stdout.split("\n")
    return sorted(short(n) for n in dem if n.strip())


def cmd_tests(stats_csv, log):
    launched = collections.Counter()
    for r in csv.DictReader(open(stats_csv)):
        launched[short(r["Name"])] += int(r["Calls"])
    allk = compiled_kernels()
    result = [ln.strip() for ln in open(log) if re.search(r"\d+ passed", ln)][-1].strip("= ")
    missing = [k for k in allk if k not in launched]
    md = ["# Kernels launched by the GPU test suite", "",
          "Every kernel instantiation compiled into `libexact.so` (%d, listed from the" % len(allk),
          "device code of `exact_kernels.hip`, `exact_tv.hip` and `exact_dense.hip`) and",
          "the number of launches the GPU tests make of it.",
          ("No instantiation is left unlaunched: each runs in at least one GPU test\n"
           "whose results are checked.") if not missing else
          "Not launched: %s." % ", ".join(missing), "",
          "Command (from the repository root, TMPDIR=/tmp, `<out>` an output",
          "directory):", "", "```", TESTS_TRACE, "```", "",
          "Summarised by `python -m paper_2503_19925_amd.profsum tests "
          "<out>/prof_tests/tests_kernel_stats.csv <out>/tests_traced.log`.", "",
          "Result: %s." % result, "", "| kernel | launches |", "|---|---|"]
    md += ["| %s | %d |" % (k, launched.get(k, 0)) for k in allk]
    other = sorted(set(launched) - set(allk))
    md += ["", "Other kernels in the trace (runtime copies and fills, torch): %d kinds." % len(other)]
    with open(os.path.join(PROFILES, "kernels_gpu_tests.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("wrote kernels_gpu_tests.md; %d compiled, %d not launched" % (len(allk), len(missing)))


# ------------------------------------------------------------- batched leg

def step_kind(name):
    """The step kernel a dispatch belongs to (batched or single-scan), or
    None."""
    n = short(name)
    for k in ("kb_forward", "kb_back_update", "kb_finish", "k_forward", "k_back_update",
              "k_eg_finish"):
        if n == k or n.startswith(k + "<"):
            return k
    return None


def cmd_batched(trace_csv, err_log, out=None):
    out = out or os.path.join(PROFILES, "kernels_batched.md")
    rows = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
                  for r in csv.DictReader(open(trace_csv)))
    err = open(err_log).read()
    t_ser = float(re.search(r"serial: ([0-9.]+) s", err).group(1))
    t_bat = float(re.search(r"batched: ([0-9.]+) s", err).group(1))
    kb = [r for r in rows if (step_kind(r[2]) or "").startswith("kb_")]
    t0, t1 = kb[0][0], kb[-1][1]
    phase = [r for r in rows if r[0] >= t0 and r[1] <= t1]
    busy = sum(b - a for a, b, _ in phase)
    per = collections.defaultdict(lambda: [0, 0])
    for a, b, n in phase:
        per[short(n)][0] += 1
        per[short(n)][1] += b - a
    # steps: each batched step ends with its kb_finish
    steps, cur, start = [], collections.Counter(), None
    for a, b, n in kb:
        start = a if start is None else start
        cur[step_kind(n)] += b - a
        if step_kind(n) == "kb_finish":
            steps.append((start, b, cur))
            cur, start = collections.Counter(), None
    ser = collections.defaultdict(lambda: [0, 0])
    for a, b, n in rows:
        k = step_kind(n)
        if b < t0 and k in ("k_forward", "k_back_update", "k_eg_finish"):
            ser[k][0] += 1
            ser[k][1] += b - a
    md = ["# Kernel times of the batched leg (64 scans to natural residual 1e-4)", "",
          "The benchmark's batched leg alone: 64 uneven scans (N in {128..768}, 30-360",
          "views, 10-64 energy bins, 2-4 windows; seed 401), each solved to rho <= 1e-4",
          "one at a time (serial) and then all together in one batch.  Command (from",
          "the repository root, TMPDIR=/tmp; the raw trace is not kept):", "",
          "```", BATCHED_TRACE, "```", "",
          "Summarised by `python -m paper_2503_19925_amd.profsum batched "
          "<trace dir>/b_kernel_trace.csv <bench stderr> <out.md>`.", "",
          "Wall time in this (profiled) run: serial %.2f s, batched %.2f s.  The profiler" % (
              t_ser, t_bat),
          "adds a cost to every dispatch, and the serial leg makes about 40 times as many",
          "as the batched one, so these walls are not the benchmark's; the kernel times",
          "below are the comparison.", "",
          "**Batched phase** (first to last batched kernel): %.3f s, of which kernels %.3f s "
          "(%.1f %% busy), %d dispatches, %d steps." % (
              (t1 - t0) / 1e9, busy / 1e9, 100.0 * busy / (t1 - t0), len(phase), len(steps)), "",
          "| kernel | calls | avg (us) | total (s) |", "|---|---|---|---|"]
    for k, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        md.append("| %s | %d | %.2f | %.3f |" % (k, c, t / c / 1e3, t / 1e9))
    md += ["", "Per batched step, by share of the steps (scans drop out as they converge):",
           "", "| steps | time (s) | per step (us) | forwards (us) | back + update (us) |",
           "|---|---|---|---|---|"]
    n = len(steps)
    for lo, hi in ((0, 0.5), (0.5, 0.8), (0.8, 0.9), (0.9, 1.0)):
        seg = steps[int(lo * n):int(hi * n)]
        if not seg:
            continue
        tot = sum(b - a for a, b, _ in seg)
        fw = sum(c.get("kb_forward", 0) for _, _, c in seg)
        bu = sum(c.get("kb_back_update", 0) for _, _, c in seg)
        md.append("| %d-%d | %.3f | %.1f | %.1f | %.1f |" % (
            int(lo * n), int(hi * n), tot / 1e9, tot / len(seg) / 1e3, fw / len(seg) / 1e3,
            bu / len(seg) / 1e3))
    md += ["", "**Serial leg's kernels** (every single-scan step kernel before the batched "
           "phase; the run's few other solve_512 steps are among them):", "",
           "| kernel | calls | avg (us) | total (s) |", "|---|---|---|---|"]
    for k in ("k_forward", "k_back_update", "k_eg_finish"):
        if k in ser:
            c, t = ser[k]
            md.append("| %s | %d | %.2f | %.3f |" % (k, c, t / c / 1e3, t / 1e9))
    per_kind = collections.Counter()
    for a, b, nme in phase:
        per_kind[step_kind(nme)] += b - a
    md += ["", "Batched against serial kernel time: forwards %.2fx, back-projection + "
           "update %.2fx." % (ser["k_forward"][1] / max(per_kind["kb_forward"], 1),
                              ser["k_back_update"][1] / max(per_kind["kb_back_update"], 1))]
    with open(out, "w") as f:
        f.write("\n".join(md) + "\n")
    print("wrote", out)


def cmd_batched_counters(counter_csv, out=None):
    out = out or os.path.join(PROFILES, "counters_batched.md")
    per = collections.defaultdict(dict)        # dispatch -> counter -> value
    meta = {}
    for r in csv.DictReader(open(counter_csv)):
        k = step_kind(r["Kernel_Name"])
        if k not in ("kb_forward", "kb_back_update"):
            continue
        d = r["Dispatch_Id"]
        per[d][r["Counter_Name"]] = float(r["Counter_Value"])
        meta[d] = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]), k)
    rows = sorted((meta[d][0], meta[d][1], meta[d][2], per[d]) for d in per)
    md = ["# VALU issue of the batched kernels (hardware counters)", "",
          "One rocprofv3 counter pass over the benchmark's batched leg alone (64 uneven",
          "scans to rho <= 1e-4 in one batch, without the one-at-a-time pass).  Command",
          "(from the repository root, TMPDIR=/tmp):", "", "```", BATCHED_PMC, "```", "",
          "Summarised by `python -m paper_2503_19925_amd.profsum batched_counters "
          "<run dir>/run_counter_collection.csv <out.md>`.", "",
          "Fractions as in `counters_utilisation.md` (1024 SIMDs at the published 2.4 GHz,",
          "the dispatch's own duration from the counter run; VALU issue at 2 cycles per",
          "instruction, and at 4), time-weighted over the dispatches of each kind.  Early",
          "dispatches hold all 64 scans' work; later ones fewer, as scans converge.", "",
          "| kernel | dispatches | part of the run (by dispatch order) | mean duration (us) | VALU issue "
          "| VALU at 4 cycles | waves / SIMD |", "|---|---|---|---|---|---|---|"]
    for k in ("kb_forward", "kb_back_update"):
        rs = [r for r in rows if r[2] == k]
        n = len(rs)
        for lo, hi in ((0.0, 0.5), (0.5, 0.8), (0.8, 1.0), (0.0, 1.0)):
            seg = rs[int(lo * n):int(hi * n)]
            if not seg:
                continue
            cyc = sum((b - a) for a, b, _, _ in seg) * 1e-9 * CLOCK_GHZ * 1e9
            valu = sum(c.get("SQ_INSTS_VALU", 0.0) for _, _, _, c in seg)
            wc = sum(c.get("SQ_WAVE_CYCLES", 0.0) for _, _, _, c in seg)
            md.append("| %s | %d | %d-%d %% | %.1f | %.0f %% | %.0f %% | %.1f |" % (
                k, len(seg), round(100 * lo), round(100 * hi),
                sum((b - a) for a, b, _, _ in seg) / len(seg) / 1e3,
                100 * valu * 2 / SIMDS / cyc, 100 * valu * 4 / SIMDS / cyc,
                wc * 4 / SIMDS / cyc))
    with open(out, "w") as f:
        f.write("\n".join(md) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    a = sys.argv[1:]
    if a[:1] == ["counters"] and len(a) == 3:
        cmd_counters(a[1], a[2])
    elif a[:1] == ["kernels"] and len(a) == 2:
        cmd_kernels(a[1])
    elif a[:1] == ["utilisation"] and len(a) == 2:
        cmd_utilisation(a[1])
    elif a[:1] == ["tests"] and len(a) == 3:
        cmd_tests(a[1], a[2])
    elif a[:1] == ["batched_counters"] and len(a) in (2, 3):
        cmd_batched_counters(a[1], a[2] if len(a) == 3 else None)
    elif a[:1] == ["batched"] and len(a) in (3, 4):
        cmd_batched(a[1], a[2], a[3] if len(a) == 4 else None)
    else:
        raise SystemExit(__doc__)
