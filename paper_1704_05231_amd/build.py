"""Builds libgabor.so in-tree with hipcc for gfx950.

    python -m paper_1704_05231_amd.build

All HIP code is compiled with packed-FP32 instruction selection disabled; the
scalar and float2 FP32 code is left to the compiler's ordinary VALU lowering.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgabor.so")

# (source, extra defines, object name): the fused kernel is built once per
# arithmetic form so that its objects compile in parallel.
SOURCES = ([("gabor_plan.cpp", [], "gabor_plan"), ("gabor_lsdft.cpp", [], "gabor_lsdft"),
            ("gabor_batch.cpp", [], "gabor_batch"),
            ("gabor_fp32.hip", [], "gabor_fp32"), ("gabor_adjoint.hip", [], "gabor_adjoint"),
            ("gabor_iir.hip", [], "gabor_iir"), ("gabor_sdft.hip", [], "gabor_sdft"),
            ("gabor_noalloc.hip", [], "gabor_noalloc")]
           + [("gabor_fused.hip", [f"-DGABOR_FORM={k}"], f"gabor_fused_{k}") for k in range(5)]
           + [("gabor_ws.hip", [f"-DGABOR_FORM={k}"], f"gabor_ws_{k}") for k in range(5)])
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; libgabor needs ROCm's hipcc to build")


_HARMLESS = "'-packed-fp32-ops' is not a recognized feature for this target"


def _run(cmd, verbose):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if _HARMLESS not in ln]
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), flush=True)


def build(verbose: bool = False) -> str:
    objs = []
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-Wall"]
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    cmds = []
    for src, defs, name in SOURCES:
        obj = os.path.join(obj_dir, name + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([hipcc()] + flags + defs + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1)))
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for fut in [ex.submit(_run, cmd, verbose) for cmd in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    _run(cmd, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
