"""Measurement helpers run on the GPU machine (not part of the solver path).

    python -m paper_2502_12620_amd.measure copy  [--mb 1024]
        a plain device-to-device copy of known size, the calibration kernel
        for the FETCH_SIZE / WRITE_SIZE counters;
    python -m paper_2502_12620_amd.measure sweep [--steps 10]
        the roofline sweep: uniform 2-D and 3-D vortex forests large enough
        to live in HBM (above the 256 MB last-level cache), FP64 stage kernel
        timed with HIP events around each launch.

Each prints JSON lines.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import torch

from . import dgamr as G
from . import workloads as W

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# estimated FP64 flops per DOF per stage (volume evaluate + flux + project,
# face traces + Rusanov + lift), by (dim, degree)
FLOP_PER_DOF = {(2, 1): 76, (2, 2): 120, (2, 3): 176, (3, 1): 207, (3, 2): 480, (3, 3): 945}


def stage_bytes_per_dof(dim: int, n_cell: int) -> float:
    """Algorithmic bytes of the fused stage kernel per DOF, averaged over
    the three stages: U_s read, U_n read on stages 2-3, U_next write, face
    layer of the neighbours."""
    face = 8.0 * 2 * dim / n_cell
    return (16.0 + 24.0 + 24.0) / 3.0 + face


def run_workload(w, steps: int, warmup: int = 3, precision=G.FP64, variant=-1):
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma, precision=precision)
    f.set_tuning(G.TUNE_STAGE_VARIANT, variant)
    u = f.project_ic(G.IC_VORTEX, w.ic_params)
    work = f.new_work()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    f.run(u, work, dt, warmup, w.cfl)
    torch.cuda.synchronize()
    f.profile_enable(True)
    t0 = time.perf_counter()
    f.run(u, work, dt, steps, w.cfl)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    f.profile_enable(False)
    ms, launches = f.profile_read()
    n = f.n_leaves
    dof = w.dofs(n)
    avg = ms / 1e3 / launches
    bpd = stage_bytes_per_dof(w.dim, w.n_cell)
    gbs = dof * bpd / avg / 1e9
    flops = FLOP_PER_DOF[(w.dim, w.degree)] * dof / avg / 1e12
    bad = f.check_state(u, work)
    del f, u, work
    torch.cuda.empty_cache()
    return {"workload": w.name, "precision": "fp32" if precision == G.FP32_MFMA else "fp64", "variant": variant,
            "dim": w.dim, "degree": w.degree, "leaves": n, "dofs": dof,
            "state_MB": dof * 8 / 1e6, "steps": steps, "dof_stage_per_s": dof * 3 * steps / el,
            "stage_kernel_us": avg * 1e6, "algorithmic_bytes_per_dof": bpd, "achieved_GBs": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "est_TFLOPs": flops, "fp64_frac": flops / FP64_PEAK_TFLOPS,
            "nonphysical_cells": bad}


def cmd_sweep(args):
    cases = [W.roofline_2d(k, p) for k in (32, 64, 128) for p in (1, 2)]
    cases += [W.roofline_2d(64, 3)]
    cases += [W.roofline_3d(16, p) for p in (1, 2)]
    for w in cases:
        if args.only and w.name not in args.only.split(","):
            continue
        prec = G.FP32_MFMA if args.precision == "fp32" else G.FP64
        variants = [0, 1] if (w.dim == 2 and args.variants and prec == G.FP64) else [-1]
        for var in variants:
            print(json.dumps(run_workload(w, args.steps, precision=prec, variant=var)), flush=True)


def cmd_copy(args):
    n = args.mb * 1024 * 1024 // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.reps
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "ms": ms,
                      "GBs_read_plus_write": 2 * n * 8 / ms / 1e6}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--steps", type=int, default=10)
    s.add_argument("--only", default="", help="comma-separated workload names")
    s.add_argument("--variants", action="store_true", help="2-D: time both stage kernels")
    s.add_argument("--precision", choices=["fp64", "fp32"], default="fp64", help="residual arithmetic")
    c = sub.add_parser("copy")
    c.add_argument("--mb", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    {"sweep": cmd_sweep, "copy": cmd_copy}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
