"""Builds the HIP library libwbsph.so for gfx950 (hipcc, in-tree)."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libwbsph.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], check=True)
    return obj


def build(jobs: int = 8) -> str:
    """Compile every .hip source and link libwbsph.so (always rebuilds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    build_example()
    return LIB


EXAMPLE = os.path.join(LIBDIR, "run_case")


def build_example() -> str:
    """The plain C caller of the library (examples/run_case.c), built with gcc
    against the HIP runtime API and linked to libwbsph.so next to it."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = EXAMPLE + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
                    "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(rocm, "include"),
                    os.path.join(HERE, "examples", "run_case.c"), "-o", tmp, "-L" + LIBDIR, "-lwbsph",
                    "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN",
                    "-Wl,-rpath," + os.path.join(rocm, "lib")], check=True)
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build())
