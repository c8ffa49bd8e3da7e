"""Build libchemora.so (gfx950) in-tree with hipcc.

Usage: ``python -m paper_1307_6488_amd.build``.  Cross-compiles without a
GPU: each translation unit (or part of one) is compiled in parallel to an object under
``_build/`` and the objects are linked into ``paper_1307_6488_amd/libchemora.so``.
Packed FP32 instructions are disabled for the whole library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libchemora.so")
# (source, defines, object): the stage kernels are built in parts -- per
# precision and per batched form -- that compile in parallel
UNITS = [
    ("chemora.hip", [], "chemora"),
    ("sync.hip", [], "sync"),
    *[("stage_o4.hip", [f"-DCHEMORA_PART_SPLIT={sp}", f"-DCHEMORA_PART_PERSIST={pe}"], f"stage_o4_s{sp}p{pe}")
      for sp in (0, 1) for pe in (0, 1)],
    *[("stage_o8.hip", [f"-DCHEMORA_PART_PERSIST={pe}"], f"stage_o8_p{pe}") for pe in (0, 1)],
]
SOURCES = sorted({u[0] for u in UNITS})
ARCH = os.environ.get("CHEMORA_ARCH", "gfx950")

# -ffp-contract=on: a multiply and an add are fused only where one source
# expression holds both (the C rule), never across statements by the code
# generator, whose choices depend on the surrounding code.  Every instance of
# the stage kernel (tile variants, single-patch, batched and persistent
# forms) then computes the same bits for a point.
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _compile(unit, extra, verbose: bool) -> str:
    src, defines, name = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, *defines, *extra, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src),
           "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), flush=True)
    return obj


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(lambda u: _compile(u, list(extra), verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
