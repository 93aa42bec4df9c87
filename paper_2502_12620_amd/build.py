"""Build the HIP library libdgamr.so for gfx950 (in-tree, hipcc)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgamr.so")
OBJDIR = os.path.join(HERE, "_build")

HIP_SOURCES = ["dgamr_api.hip", "pool_api.hip", "static_api.hip"]
CXX_SOURCES = ["forest.cpp"]
# degree-templated kernels: one translation unit per (dim, degree, part);
# the parts split the heavy kernels of one (dim, degree) pair (csrc/inst.hip)
INSTANCES = [(d, p, part) for d in (2, 3) for p in (0, 1, 2, 3) for part in (0, 1, 2, 3, 4)]

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fconstexpr-steps=200000000",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
    "-I" + os.path.join(HERE, "..", "include"),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd[:3]) + " ...")
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    objs_keep = []
    for s in HIP_SOURCES:
        o = os.path.join(OBJDIR, s + ".o")
        jobs.append(["hipcc", *HIPFLAGS, "-c", os.path.join(CSRC, s), "-o", o])
    # DGAMR_BUILD_ONLY="2_2,api" recompiles only those units and relinks the
    # existing objects of the others (a development shortcut; the default
    # compiles everything)
    only = [x for x in os.environ.get("DGAMR_BUILD_ONLY", "").split(",") if x]
    for d, p, part in INSTANCES:
        o = os.path.join(OBJDIR, f"inst_{d}_{p}_{part}.o")
        if only and f"{d}_{p}" not in only and f"{d}_{p}_{part}" not in only and os.path.exists(o):
            objs_keep.append(o)
            continue
        jobs.append(["hipcc", *HIPFLAGS, f"-DDG_D={d}", f"-DDG_P={p}", f"-DDG_PART={part}", "-c",
                     os.path.join(CSRC, "inst.hip"), "-o", o])
    for s in CXX_SOURCES:
        o = os.path.join(OBJDIR, s + ".o")
        jobs.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
                     "-I/opt/rocm/include", "-c", os.path.join(CSRC, s), "-o", o])
    # longest first: the 3-D high-degree units dominate
    jobs.sort(key=lambda j: ("-DDG_D=3" in j, "-DDG_P=3" in j, "-DDG_P=2" in j), reverse=True)
    with ThreadPoolExecutor(max_workers=min(int(os.environ.get("MAX_JOBS", "8")), len(jobs))) as ex:
        logs = list(ex.map(_run, jobs))
    if verbose:
        for l in logs:
            sys.stderr.write(l)
    objs = [j[-1] for j in jobs] + objs_keep
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
