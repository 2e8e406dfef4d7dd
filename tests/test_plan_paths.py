"""The planner's closed-form Partition path against its weight-array path
(host code of libfim.so, no GPU): tests/plan_equivalence.cpp, built with
hipcc against the library."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2108_05038_amd")


def test_closed_form_partition_matches_weight_arrays(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    lib = os.path.join(PKG, "libfim.so")
    if not hipcc or not os.path.exists(lib):
        pytest.skip("hipcc or the built library is missing")
    exe = str(tmp_path / "plan_equivalence")
    cmd = [hipcc, "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(PKG, "csrc"), os.path.join(ROOT, "tests", "plan_equivalence.cpp"),
           "-o", exe, "-L" + PKG, "-lfim", "-Wl,-rpath," + PKG]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "mismatching trials: 0" in r.stdout
