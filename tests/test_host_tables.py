"""Host logic of the forward projector's tables, checked on the CPU.

tests/host_tables_check.cpp includes the library's own table code
(paper_2503_19925_amd/csrc/exact_tables.h) and checks it against brute
force: every (ray, line) with a positive tap weight on an image pixel lies
inside its block's line range, on 401 random and workload-sized
parallel-beam geometries (views along and across the axes, at 45 degrees,
bins of 0.3 to 2.7 pixels); and the workgroup dispatch order is a
permutation for 3000 random weight lists, CU counts and slots per CU.  The
harness is host code only: it is compiled with hipcc (for the HIP headers
the table code includes) and makes no GPU call.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_forward_tables_against_brute_force(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc is not available")
    exe = str(tmp_path / "host_tables_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-w",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2503_19925_amd", "csrc"),
           os.path.join(ROOT, "tests", "host_tables_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("OK"), res.stdout
