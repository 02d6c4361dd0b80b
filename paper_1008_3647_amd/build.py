"""Build libufg.so for gfx950 with hipcc (in-tree, next to this file), then
the plain-C example program examples/solve_from_c against it.

Usage: python -m paper_1008_3647_amd.build [--jobs N] [--debug]
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libufg.so")
EXAMPLES = os.path.join(HERE, "examples")
SOURCES = ["api.cpp", "ops.cpp", "solvers.cpp", "split.cpp", "batched.hip", "hop.hip",
           "hop_stream.hip", "temporal.hip", "krylov.hip", "noalloc.hip",
           "hmc.hip", "lowd.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(debug: bool = False):
    f = ["-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off (see DESIGN notes on gfx950 codegen)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    f += ["-O1", "-g"] if debug else ["-O3"]
    return f


def compile_one(src: str, debug: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *flags(debug), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 8, debug: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    build_c_example(verbose)
    return LIB


def build_c_example(verbose: bool = True) -> str:
    """Compile examples/solve_from_c.c with gcc as C11 against include/ufg.h and
    libufg.so (run path: the package directory, then ROCm's libraries)."""
    inc = os.path.join(os.path.dirname(HERE), "include")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out = os.path.join(EXAMPLES, "solve_from_c")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{inc}", f"-I{rocm}/include", os.path.join(EXAMPLES, "solve_from_c.c"),
           "-o", out + ".tmp", f"-L{HERE}", "-lufg", f"-L{rocm}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/..", f"-Wl,-rpath,{rocm}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C example failed to build\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(out + ".tmp", out)
    if verbose:
        print(f"built {out}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.debug)


if __name__ == "__main__":
    sys.exit(main())
