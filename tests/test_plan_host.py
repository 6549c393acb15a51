"""Host checks of the symbolic plan (no device).

tests/plan_check.cpp is built with g++ against the library's plan.cpp and
run: for several lateral grids, panel depths and leaf sizes it checks the
elimination order, the push and pull maps of the extend-add between each
child and its parent front (Sec. 2.1-2.2), the map by which a first child's
contributions join its parent's right-hand side (one writer per entry), and
that the per-front storage regions tile their buffers.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1204_0111_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_invariants_hold(tmp_path):
    exe = str(tmp_path / "plan_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "plan_check.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and "FAIL" not in out.stdout, out.stdout
    assert out.stdout.count("ok ") == 7, out.stdout
