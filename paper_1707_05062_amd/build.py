"""Build the gfx950 shared library ``libkohler.so`` in-tree with hipcc.

Each source is compiled to an object of its own (in parallel), then the objects are linked.

Usage: python -m paper_1707_05062_amd.build [--phase-clock]

--phase-clock builds ``libkohler_phase.so`` instead: the same library with per-workgroup phase
timestamps recorded by the curve kernel (see ``phase_clock.py``); it is never loaded by default.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libkohler.so")
PHASE_LIB = os.path.join(PKG, "libkohler_phase.so")
ROOFLINE_LIB = os.path.join(PKG, "libkohler_roofline.so")
ROOFLINE_SOURCE = "kohler_roofline.hip"

SOURCES = ["kohler_kernels.hip", "kohler_api.cpp", "kohler_server.cpp", "kohler_segment.hip", "kohler_noalloc.hip"]
HEADERS = ["kohler_impl.h", "kohler_host.h", "kohler_arena.h", "kohler_columns.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every uniform-address atomic here is issued by a single lane; the wave-aggregation rewrite
    # would only add a wait for the result right after issue
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _jobs() -> int:
    try:
        return max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1))
    except ValueError:
        return 1


def build(out: str = LIB, verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every HIP/C++ source and link them into one shared library (always recompiles)."""
    objdir = out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    flags = [*HIPCC_FLAGS, *(extra or []), f"-I{INCLUDE}", f"-I{CSRC}"]

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *flags, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_roofline(verbose: bool = False) -> str:
    """The benchmark's roofline probes (HBM read stream, LDS atomic rates): a library of their own."""
    tmp = ROOFLINE_LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-shared", "-o", tmp, os.path.join(CSRC, ROOFLINE_SOURCE)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, ROOFLINE_LIB)
    return ROOFLINE_LIB


def build_phase_clock(verbose: bool = False) -> str:
    """The library with the curve kernel's phase timestamps compiled in (a measurement build)."""
    return build(PHASE_LIB, verbose=verbose, extra=["-DKOHLER_PHASE_CLOCK=1"])


def is_stale(out: str = LIB) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(INCLUDE, "kohler.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    if "--phase-clock" in sys.argv[1:]:
        print(build_phase_clock(verbose=True), file=sys.stderr)
    elif "--roofline" in sys.argv[1:]:
        print(build_roofline(verbose=True), file=sys.stderr)
    else:
        print(build(verbose=True), file=sys.stderr)
        print(build_roofline(verbose=True), file=sys.stderr)
