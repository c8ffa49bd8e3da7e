"""The stage kernel's LDS staging layouts, checked on the host.

tests/layout_check.hip includes the kernel header itself (its layout types
are host-and-device constexpr code) and checks, for every tile variant's
layout (one plane and the z-depth variants, orders 4 and 8) over ragged
patches: that a work-item's every stencil tap decodes back to the point it
stands for and lies inside the staged buffer, and that the clamped global
staging offsets of every tile stay inside the patch's stored box (pairs of
doubles inside one row).  No GPU is involved.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_staging_layouts_are_consistent_and_in_bounds(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "layout_check")
    cmd = [hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1307_6488_amd", "csrc"),
           os.path.join(ROOT, "tests", "layout_check.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "0 violations" in r.stdout, r.stdout + r.stderr
