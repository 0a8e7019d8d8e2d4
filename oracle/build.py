"""Compile the C reference (lb_oracle.c, the library's C ABI on host
pointers) into oracle/_lib/liblb_oracle.so with the system C compiler.

TEST INFRASTRUCTURE ONLY: nothing in the product path loads it.

    python -m oracle.build
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "_lib", "liblb_oracle.so")


def build(verbose=False):
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("a C compiler is required to build %s" % LIB)
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    # plain IEEE double arithmetic: no fast-math, no FMA contraction
    # OpenMP over sites: per-site arithmetic is the same on any thread
    cmd = [cc, "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp", SRC, "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("C compiler failed building %s" % LIB)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
