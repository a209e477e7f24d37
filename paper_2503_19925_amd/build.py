"""Builds libexact.so (HIP for gfx950) in the package directory.

    python -m paper_2503_19925_amd.build

Flags: gfx950 only; packed-FP32 instruction selection disabled (some forms
have produced wrong results on these parts); floating-point contraction off
so that every fused multiply-add in the kernels is an explicit fma/fmaf
(the projector weights must be bit-identical in the forward and the
back-projector).  The kernels' tile knobs come from tuned.json, which the
autotuner (tune.py) writes; without it the sources' defaults apply.
"""
import hashlib
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libexact.so")
TUNED = os.path.join(HERE, "tuned.json")
SOURCES = ["csrc/exact_kernels.hip", "csrc/exact_tv.hip", "csrc/exact_dense.hip",
           "csrc/exact_capi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]

# compile-time knobs of exact_kernels.hip that the autotuner chooses, with
# the sources' defaults
DEFAULT_KNOBS = {"EXACT_LINE_BATCH": 4, "EXACT_VIEW_BATCH": 4, "EXACT_FWD_SEGS": 4}
KNOBS = tuple(sorted(DEFAULT_KNOBS))


def tuned_knobs():
    """The knob values to build with: tuned.json's where it sets them, the
    sources' defaults elsewhere."""
    knobs = dict(DEFAULT_KNOBS)
    try:
        rec = json.load(open(TUNED))
    except (OSError, ValueError):
        return knobs
    knobs.update({k: int(v) for k, v in rec.get("knobs", {}).items() if k in KNOBS})
    return knobs


def defines(knobs):
    return ["-D%s=%d" % (k, knobs[k]) for k in sorted(knobs)]


# sources whose text decides what the step's kernels do (the kernels, the
# shared declarations, and the host code that builds the kernels' tables and
# work lists)
KERNEL_SOURCES = ["csrc/exact_kernels.hip", "csrc/exact_internal.h", "csrc/exact_capi.hip",
                  "csrc/exact_tables.h"]


def build_id(knobs=None):
    """SHA-1 of the kernel sources and the knob values they are compiled with:
    what a stored hardware-counter reading is valid for."""
    knobs = tuned_knobs() if knobs is None else knobs
    h = hashlib.sha1()
    for src in KERNEL_SOURCES:
        h.update(open(os.path.join(HERE, src), "rb").read())
    h.update(" ".join(defines(knobs)).encode())
    return h.hexdigest()


def build(verbose=False, out=LIB, knobs=None):
    """Compiles the library into `out` with the given knob values (default:
    tuned.json's)."""
    knobs = tuned_knobs() if knobs is None else knobs
    tmp = out + ".tmp"
    cmd = [HIPCC] + FLAGS + defines(knobs) + [
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"), "-o", tmp] + [
        os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
