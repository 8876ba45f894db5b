"""Build the HIP library (gfx950) in-tree: paper_2201_06620_amd/librosnet.so.

Every source is compiled to an object of its own (in parallel), then the
objects are linked into one shared library.  Always recompiles."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librosnet.so")
SOURCES = ["gemm_f32_4m.hip", "gemm_f64.hip", "gemm_bf16x3.hip", "gemm_f32_3m.hip",
           "kernels.hip", "api.cpp", "plan.cpp", "network.cpp", "batch.cpp", "serve.cpp",
           "stream.cpp", "noalloc.hip"]
ARCH = os.environ.get("RN_OFFLOAD_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Wno-unused-result", "-pthread",
         # Packed FP32 instructions stay off: hipcc would otherwise form
         # v_pk_* ops from plain float code.
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    objs, pending, failed = [], [], []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [hipcc] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        while len(pending) >= jobs:
            failed += _reap(pending, block=True)
        pending.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                              stderr=subprocess.STDOUT, text=True)))
    while pending:
        failed += _reap(pending, block=True)
    if failed:
        for src, out in failed:
            sys.stderr.write(f"--- {src}\n{out}")
        raise RuntimeError("hipcc failed: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


def _reap(pending, block):
    """Wait for the oldest compile; return [(source, output)] if it failed."""
    src, p = pending.pop(0)
    out, _ = p.communicate()
    if p.returncode != 0:
        return [(src, out)]
    return []


if __name__ == "__main__":
    print(build(verbose=True))
