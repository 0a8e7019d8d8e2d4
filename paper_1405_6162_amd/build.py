"""Compile the gfx950 HIP library (liblb.so) in-tree with hipcc, and the
plain-C example program (lb_example) next to it.

    python -m paper_1405_6162_amd.build

The library is written for gfx950 only; packed-FP32 instruction selection is
switched off (hipcc forms v_pk_*_f32 on its own from scalar float code).
"""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "lb_api.hip")
DEPS = [os.path.join(PKG, "csrc", n) for n in ("d3q19.h", "kernels.h")] + [os.path.join(ROOT, "include", "lb.h")]
LIB_DIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIB_DIR, "liblb.so")
EXAMPLE_SRC = os.path.join(PKG, "csrc", "lb_example.c")
EXAMPLE = os.path.join(LIB_DIR, "lb_example")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build liblb.so")
    return exe


def build(verbose=False):
    """Compile liblb.so (always recompiles).  Returns the library path."""
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % LIB)
    os.replace(tmp, LIB)
    build_example(verbose)
    return LIB


def build_example(verbose=False):
    """The plain-C example (lb_example.c) linked against liblb.so and the HIP
    runtime, next to the library."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("a C compiler is required to build %s" % EXAMPLE)
    tmp = EXAMPLE + ".tmp%d" % os.getpid()
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), EXAMPLE_SRC, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-L", LIB_DIR, "-llb", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("C compiler failed building %s" % EXAMPLE)
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
