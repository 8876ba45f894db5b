"""Build the HIP library (gfx950) in-tree: paper_2201_06620_amd/librosnet.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librosnet.so")
SOURCES = ["kernels.hip", "api.cpp", "plan.cpp", "network.cpp", "batch.cpp", "serve.cpp",
           "stream.cpp"]
ARCH = os.environ.get("RN_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    """Compile every source into one shared library (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-result", "-pthread",
           # Packed FP32 instructions stay off: hipcc would otherwise form
           # v_pk_* ops from plain float code.
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
