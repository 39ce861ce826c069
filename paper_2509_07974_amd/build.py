"""Build libfpcf4.so for gfx950 with hipcc (in-tree).

    python -m paper_2509_07974_amd.build        # or __graft_entry__.build()

Every HIP source is compiled to an object under ``_build/`` (in parallel;
stage_a.hip once per supported nmax so its large unrolled kernels compile
concurrently) and linked into ``paper_2509_07974_amd/libfpcf4.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfpcf4.so")
NMAX_SUPPORTED = 16

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed fp32 VALU ops are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _torch_lib_dir():
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return None


def _jobs():
    hip = _hipcc()
    jobs = []
    for src in ("api.hip", "cells.hip", "stage_b.hip", "stage_b_pairs.hip", "natural.hip",
                "threepcf.hip", "sort.hip", "stage_a.hip"):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        jobs.append([hip, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    for n in range(NMAX_SUPPORTED + 1):
        obj = os.path.join(BUILD, f"stage_a_n{n:02d}.o")
        jobs.append([hip, *FLAGS, f"-DFPCF4_STAGE_A_N={n}", "-c",
                     os.path.join(CSRC, "stage_a.hip"), "-o", obj])
    return jobs


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "not a recognized feature" not in l)
    return r.returncode, cmd[-1], err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    cmds = _jobs()
    objs = [c[-1] for c in cmds]
    with cf.ThreadPoolExecutor(jobs) as ex:
        for rc, obj, err in ex.map(_run, cmds):
            if verbose and err.strip():
                print(err, file=sys.stderr)
            if rc != 0:
                raise RuntimeError(f"hipcc failed for {obj}:\n{err}")
    tmp = LIB + ".tmp"
    # One HIP runtime per process: resolve libamdhip64.so.7 from PyTorch's
    # bundled ROCm first (PyTorch supplies the device memory and streams this
    # library runs on), then from the system ROCm.
    rpath = [d for d in (_torch_lib_dir(), "/opt/rocm/lib") if d]
    hiplib = os.path.join(rpath[0], "libamdhip64.so")
    link = ["g++", "-shared", "-fPIC", "-o", tmp, *objs,
            *[f"-Wl,-rpath,{d}" for d in rpath], "-Wl,--enable-new-dtags",
            hiplib, "-Wl,--no-undefined"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
