"""Compiles libmoss.so for gfx950 with hipcc (in-tree, under _build/), and the
scenario generator's host helper libscen.so with gcc.

Flags: no FP contraction (the op order is part of the model's definition),
correctly rounded FP32 divide/sqrt, denormals kept, and packed-FP32
instructions disabled.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libmoss.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("moss_api.hip", "moss_kernels.hip", "moss_mlp.hip")]
ARCH = os.environ.get("MOSS_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-fno-gpu-flush-denormals-to-zero",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


SCEN_LIB = os.path.join(BUILD, "libscen.so")
SCEN_SRC = os.path.join(HERE, "csrc", "scen_routes.c")


def build_scen(verbose: bool = False) -> str:
    """Host helper of the scenario generator (shortest-path routes; gcc,
    OpenMP)."""
    os.makedirs(BUILD, exist_ok=True)
    tmp = SCEN_LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", "-o", tmp,
           SCEN_SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SCEN_LIB)
    return SCEN_LIB


def ensure_scen() -> str:
    if not os.path.exists(SCEN_LIB):
        build_scen()
    return SCEN_LIB


def build(verbose: bool = False) -> str:
    build_scen(verbose)
    os.makedirs(BUILD, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
