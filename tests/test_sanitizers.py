"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (CPU only).

The oracle (oracle/oracle.c) and the library's host planner (the .cpp
sources: planning, pair lists, footprints, batch, streamed and network
plans) are rebuilt with gcc/g++ -fsanitize=address,undefined and driven over
seeded random shapes, grids, ranks up to 64 and invalid arguments by the
drivers in tests/sanitize/.  Any out-of-bounds access, use after free or
undefined behaviour aborts the driver; a wrong status makes it exit nonzero.
The GPU kernels are not part of these builds (their object files come from
the regular build, unsanitized, and no kernel is launched)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_06620_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2201_06620_amd", "_build")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

def _sources():
    from paper_2201_06620_amd import build as hipbuild
    return hipbuild.SOURCES


HOST = [os.path.splitext(s)[0] for s in _sources() if s.endswith(".cpp")]
KERNEL_OBJS = [os.path.splitext(s)[0] for s in _sources() if s.endswith(".hip")]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    run(["gcc", "-std=c99", "-ffp-contract=off"] + SAN +
        [os.path.join(ROOT, "oracle", "oracle.c"),
         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    r = run([exe], env=ENV, timeout=600)
    assert "ok" in r.stdout


def test_host_planner_under_sanitizers(tmp_path):
    if not all(os.path.exists(os.path.join(OBJ, o + ".o")) for o in KERNEL_OBJS):
        from paper_2201_06620_amd import build as hipbuild
        hipbuild.build()
    objs = []
    procs = []
    for src in HOST:
        o = str(tmp_path / (src + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen(
            ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN +
            ["-c", os.path.join(CSRC, src + ".cpp"), "-o", o],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    drv = str(tmp_path / "plan_driver.o")
    procs.append(subprocess.Popen(
        ["g++", "-std=c++17"] + SAN +
        ["-c", os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"), "-o", drv],
        stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-4000:]
    exe = str(tmp_path / "plan_san")
    run(["g++", "-fsanitize=address,undefined", drv] + objs +
        [os.path.join(OBJ, o + ".o") for o in KERNEL_OBJS] +
        ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-pthread", "-o", exe])
    r = run([exe], env=ENV, timeout=600)
    assert "ok" in r.stdout
