"""Build libtpcf.so in place: HIP kernels for gfx950 plus the host library.

    python -m paper_1204_6630_amd.build

Kernels: hipcc --offload-arch=gfx950 -O3, contraction off (the FP64 dot
product must stay unfused), packed FP32 instructions disabled.  Host code:
g++ -O2, contraction off and no math builtins, so sin, cos and acos stay
plain libm calls (the counting rule is defined by them).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtpcf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]
HOST_FLAGS = [
    "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin",
    "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
    "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function", "-pthread",
]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(out_dir: str | None = None, verbose: bool = True) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    k_obj = os.path.join(bdir, "kernels.o")
    _run([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", k_obj])
    objs.append(k_obj)
    for src in ("edges.cpp", "capi.cpp"):
        o = os.path.join(bdir, src.replace(".cpp", ".o"))
        _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
          "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", "-pthread",
          "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
