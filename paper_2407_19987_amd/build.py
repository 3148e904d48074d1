"""Build step of the HOBO engine: compiles the HIP kernels and the host C++
into ``libhobo.so`` next to this file, for gfx950 only.

    python -m paper_2407_19987_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhobo.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are kept out of every device build.
NO_PK_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include")]

# (source, tag, defines): the evaluation kernel is built once per precision
# (values of the Prec enum) so that its many shapes compile in parallel, and
# so are both annealers
SOURCES = [("anneal_kernels.hip", "", []), ("anneal_block.hip", "", []), ("mlp_kernels.hip", "", []),
           ("eval_kernels.hip", "", []), ("timing.hip", "", []), ("pack.cpp", "", []), ("canon.cpp", "", []), ("results.cpp", "", []), ("tt.cpp", "", []), ("tt_kernels.hip", "", []), ("gd.cpp", "", []), ("schedule.cpp", "", []),
           ("gd_kernels.hip", "", ["-ffp-contract=off"]),  # separately rounded FP64 steps
           ("abi.cpp", "", [])] + [
    ("eval_prec.hip", f"p{p}", [f"-DHOBO_EVAL_PREC={p}"]) for p in (0, 1, 2, 3, 5)] + [
    ("anneal_block.hip", f"p{p}", [f"-DHOBO_BLOCK_PREC={p}"]) for p in (0, 1, 2, 5)] + [
    ("anneal_kernels.hip", f"p{p}", [f"-DHOBO_SLAB_PREC={p}"]) for p in (0, 1, 2, 3, 5)]


def _compile(job) -> str:
    src, tag, defs = job
    obj = os.path.join(BUILD, src + (f".{tag}" if tag else "") + ".o")
    path = os.path.join(CSRC, src)
    cmd = [HIPCC, *COMMON, *NO_PK_FP32, *defs, "-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, *NO_PK_FP32, *defs, "-x", "hip", "-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 16, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
