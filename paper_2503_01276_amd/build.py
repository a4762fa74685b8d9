"""Build the HIP library libmch.so in-tree with hipcc for gfx950.

Usage: python -m paper_2503_01276_amd.build [--debug]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmch.so")
# (source, object name, extra flags); the 2D solve kernel is compiled once per
# number of sub-blocks per axis
SOURCES = [("plan.cpp", "plan", []), ("api.cpp", "api", []), ("setup2d.hip", "setup2d", []),
           ("solve2d.hip", "solve2d", []), ("backward2d.hip", "backward2d", []), ("interp.hip", "interp", []), ("macro.hip", "macro", []), ("validate.hip", "validate", []), ("solve2d_generic.hip", "solve2d_generic", []), ("solve3d_generic.hip", "solve3d_generic", []),
           ("cells3d.hip", "cells3d", [])] + \
          [("solve2d_inst.hip", f"solve2d_s{s}", [f"-DMCH_SUB={s}"]) for s in (1, 2, 4, 8)]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # keep packed-FP32 instructions out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src, name, flags in SOURCES:
        obj = os.path.join(objdir, name + ".o")
        cmd = [hipcc(), *HIP_FLAGS, *flags, *(extra or []), "-I", os.path.join(HERE, "..", "include"),
               "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        cmds.append(cmd)
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    workers = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(run, cmds))
    for cmd, res in zip(cmds, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise subprocess.CalledProcessError(res.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
