"""Builds libphasemask.so in-tree for gfx950 with hipcc.

    python -m paper_1302_0120_amd.build          (or build() from Python)

The row/column pass source is compiled once per transform length (powers
of two 16 .. 4096, and 600, 800, 1080, 1920) in parallel; objects go to ``_build/`` at the repository root and the
shared library next to this file.
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
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libphasemask.so")
LENGTHS = (16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 600, 800, 1080, 1920)
ARCH = "gfx950"
BATCH_SCHEDULES = 2  # = kBatchSchedules in csrc/pm_common.h

# -packed-fp32-ops: keep hipcc from emitting packed FP32 instructions.
# -ffp-contract=off: the kernels spell out every fused multiply-add, so one
# formula rounds the same way in every instantiation.
HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False, jobs: int | None = None, defines=(), out: str | None = None) -> str:
    """Compile every HIP source and link the library; returns its path.

    ``defines`` are extra ``NAME=VALUE`` macros for the tuning knobs of the
    kernels (``PM_LDS_PAD``, ``PM_LDS_LINE_EXTRA``, ``PM_MAX_TWIDDLE_REGS``);
    ``out`` writes the library elsewhere (objects then go to a separate
    folder), e.g. to compare variants."""
    hipcc = _hipcc()
    flags = HIPFLAGS + [f"-D{d}" for d in defines]
    build_dir = BUILD if out is None else os.path.join(BUILD, "variant_" + "_".join(d.replace("=", "") for d in defines))
    os.makedirs(build_dir, exist_ok=True)
    lib = LIB if out is None else out
    steps = []
    for L in LENGTHS:
        obj = os.path.join(build_dir, f"pm_pass_{L}.o")
        steps.append([hipcc, *flags, f"-DPM_L={L}", "-c",
                      os.path.join(CSRC, "pm_pass.hip"), "-o", obj])
    for which in range(6):
        for sched in range(BATCH_SCHEDULES):
            steps.append([hipcc, *flags, f"-DPM_BATCH_WHICH={which}", f"-DPM_BATCH_SCHED={sched}",
                          "-c", os.path.join(CSRC, "pm_batch.hip"),
                          "-o", os.path.join(build_dir, f"pm_batch_{which}_{sched}.o")])
    steps.append([hipcc, *flags, "-c", os.path.join(CSRC, "pm_aux.hip"),
                  "-o", os.path.join(build_dir, "pm_aux.o")])
    steps.append([hipcc, *flags, "-c", os.path.join(CSRC, "pm_probe.hip"),
                  "-o", os.path.join(build_dir, "pm_probe.o")])
    steps.append([hipcc, *flags, "-x", "hip", "-c", os.path.join(CSRC, "phasemask.cpp"),
                  "-o", os.path.join(build_dir, "phasemask.o")])
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for r in ex.map(_run, steps):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    objs = [s[s.index("-o") + 1] for s in steps]
    tmp = lib + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, lib)
    return lib


TIMELINE_LIB = os.path.join(PKG, "libphasemask_timeline.so")


def build_timeline(verbose: bool = False) -> str:
    """The library with per-work-group pass timelines (csrc/pm_trace.h), for
    ``python -m paper_1302_0120_amd.pass_timeline``; a profiling build, not
    loaded by the binding unless asked for."""
    return build(verbose=verbose, defines=["PM_TIMELINE=1"], out=TIMELINE_LIB)


if __name__ == "__main__":
    if "--timeline" in sys.argv:
        print(build_timeline(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
