"""Benchmark of the block-AMR DG hot path on one MI355X.

One step = one full SSP-RK3 time step of the 2-D Euler two-level AMR vortex
workload (8x8 roots of 16x16 cells, the 12 roots near the vortex refined
once -> 100 leaves, degree 2, FP64): the CFL time step and, per stage, the
guard traces, the residual and the stage update.  The timed steps are one
launch of a HIP graph holding them: three fused stage kernels per step, the
CFL reduction folded into the previous step's last stage.

Prints one JSON line: DOF-stage updates/s over exactly --steps timed steps
(inputs resident in HBM), the roofline of the dominant kernel (the fused
stage kernel: HIP events around the timed graph launch, divided by the
stage launches in it; an eager pass with events around every launch is
reported beside it), the
same run with FP32 residual arithmetic (FP64 state), the batched
workload's batch wall time p50/p99 (512 forests, 20 steps per batch, one HIP
graph per batch, the pools of the three degrees on parallel branches)
against the same forests solved one by one, the stage kernels on forests far
larger than the last-level cache (2-D 128 x 128 roots, 3-D 16^3 roots) against
the HBM and arithmetic roofs, the oracle's rate on the host cores for a
bounded sample of the same workload (all cores and one thread, plus samples
of the 3-D blast and of a 64 x 64-root forest), and the L1 / L2 density
difference and mass drift of both GPU runs against the oracle after the same
number of steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
STAGE_SOURCES = ["kernels_2d.hpp", "kernels.hpp", "kernel_common.hpp", "dg_tables.hpp", "inst.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_12620_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_stage(w, n_leaves: int) -> dict:
    """Bytes the fused stage kernel must move, per launch, averaged over the
    three stages: read U_s, read U_n on stages 2 and 3, write U_next, and
    read the neighbours' face cells (one cell layer per block face)."""
    dof = w.dofs(n_leaves)
    face_dof = dof * 2 * w.dim / w.n_cell
    per_stage = [8 * dof + 8 * face_dof + 8 * dof,            # stage 1: a = 0, U_n not read
                 16 * dof + 8 * face_dof + 8 * dof,
                 16 * dof + 8 * face_dof + 8 * dof]
    return {"dof": dof, "bytes_per_launch": sum(per_stage) / 3.0,
            "bytes_per_dof": sum(per_stage) / 3.0 / dof}


def read_counter_traffic(workload_name: str):
    """HBM traffic per launch of the stage kernel from the committed counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_c2_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_wl = re.search(r"workload:\s*(\S+)", txt)
    if not (m_hash and m_bytes and m_wl) or m_hash.group(1) != kernel_hash() or m_wl.group(1) != workload_name:
        return None
    return float(m_bytes.group(1))


def cpu_model() -> str:
    """The host CPU's model name (lscpu), or the platform string."""
    import platform
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or platform.machine()


def _oracle_forest(O, w):
    f = O.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma)
    for rule in w.initial_refinement:
        f.adapt(rule(w, f.keys()))
    return f


def _oracle_leg(O, w, ic, threads, budget_s, limiter=False, min_steps=1):
    """Whole SSP-RK3 steps of the oracle on workload w from its initial
    state at the given thread count, until budget_s has passed (at least
    min_steps).  Regrids are not taken: the sample keeps the initial forest."""
    O.set_threads(threads)
    f = _oracle_forest(O, w)
    u = f.project_ic(ic, w.ic_params)
    dof = w.dofs(f.n_leaves)
    start = time.perf_counter()
    steps = 0
    while True:
        f.step(u, w.cfl, limiter=limiter)
        steps += 1
        el = time.perf_counter() - start
        if steps >= min_steps and el > budget_s:
            break
    return {"value": dof * 3 * steps / el, "threads": O.threads(), "steps": steps, "seconds": el,
            "leaves": f.n_leaves, "dofs": dof}


def cpu_baseline(w, n_ref_steps: int, budget_s: float, legs: bool = True):
    """The oracle (as it stands) on the host cores: whole SSP-RK3 steps of the
    same workload from the same initial state, at every core the process may
    use.  Returns the rate over at least budget_s seconds of steps, and the
    oracle state after n_ref_steps steps (the reference for the accuracy of
    the GPU results).  With legs: the same workload at one thread, and
    bounded samples of the 3-D blast workload and of the 64 x 64-root
    uniform degree-2 forest, each at all cores and at one thread."""
    import oracle as O
    from paper_2502_12620_amd import workloads as W

    ncores = len(os.sched_getaffinity(0))
    O.set_threads(ncores)
    f = _oracle_forest(O, w)
    u = f.project_ic(O.IC_VORTEX, w.ic_params)
    t0 = f.totals(u)
    dof = w.dofs(f.n_leaves)
    ref = None
    start = time.perf_counter()
    steps = 0
    while True:
        f.step(u, w.cfl)
        steps += 1
        if steps == n_ref_steps:
            ref = (u.copy(), f.totals(u))
        el = time.perf_counter() - start
        if steps >= n_ref_steps and el > budget_s:
            break
    out = {"value": dof * 3 * steps / el, "unit": "DOF-stage updates/s", "cores": O.threads(), "kind": "oracle",
           "sample": f"{steps} SSP-RK3 steps of {w.name} ({f.n_leaves} leaves, {dof} DOF) from the vortex "
                     f"initial state, {el:.1f} s",
           "cpu_model": cpu_model(), "cores_available": ncores}
    if legs:
        leg_budget = budget_s / 3.0
        c3 = W.sedov_c3()
        rs = W.roofline_2d(64, 2)
        out["legs"] = {
            f"{w.name}_1_thread": _oracle_leg(O, w, O.IC_VORTEX, 1, leg_budget),
            f"{c3.name}_{ncores}_threads": _oracle_leg(O, c3, O.IC_SEDOV, ncores, leg_budget, limiter=True),
            f"{c3.name}_1_thread": _oracle_leg(O, c3, O.IC_SEDOV, 1, leg_budget, limiter=True),
            f"{rs.name}_{ncores}_threads": _oracle_leg(O, rs, O.IC_VORTEX, ncores, leg_budget),
            f"{rs.name}_1_thread": _oracle_leg(O, rs, O.IC_VORTEX, 1, leg_budget),
            "note": "DOF-stage updates/s of whole steps (at least one) from each workload's initial state; the "
                    "blast with the limiter on, its initial 176-leaf forest, no regrid in the sample",
        }
        O.set_threads(ncores)
    return out, ref[0], ref[1], t0


def accuracy(u_gpu, tot_gpu, u_ref, tot_ref, tot0):
    """Relative L1 / L2 difference of the density coefficients against the
    oracle state, and the relative mass drift of both runs."""
    import numpy as np

    d = u_gpu[:, 0] - u_ref[:, 0]
    return {"rel_l1_density": float(np.abs(d).sum() / np.abs(u_ref[:, 0]).sum()),
            "rel_l2_density": float(np.linalg.norm(d) / np.linalg.norm(u_ref[:, 0])),
            "rel_max_all": float(np.abs(u_gpu - u_ref).max() / np.abs(u_ref).max()),
            "mass_drift_gpu": float(abs(tot_gpu[0] - tot0[0]) / abs(tot0[0])),
            "mass_drift_oracle": float(abs(tot_ref[0] - tot0[0]) / abs(tot0[0]))}


def time_path(G, w, precision, hang, steps, warmup):
    """warmup + steps SSP-RK3 steps from the vortex initial state: the
    warm-up through dgamr_run, the timed `steps` as one launch of a HIP
    graph captured beforehand (dgamr_run_capture), bracketed by HIP events;
    then an eager profiled pass of the same number of steps as a check."""
    import torch

    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma, hanging=hang,
                 precision=precision)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    u = f.project_ic(G.IC_VORTEX, w.ic_params)
    work = f.new_work()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    f.run(u, work, dt, warmup, w.cfl)
    graph = f.capture_run(u, work, dt, steps, w.cfl)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()  # HIP events on the stream the graph (and so every stage kernel) runs on
    graph.launch()
    e1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the stage kernels are 3 * steps of the graph's 3 * steps + 3 launches
    # (the CFL prologue: two reductions and a slot write, a few microseconds
    # in all), so the graph's event time over 3 * steps bounds the stage
    # kernel's average duration from above
    graph_ms = e0.elapsed_time(e1)
    # cross-check: the same steps once more eagerly (continuing from the
    # timed state) with HIP events around every stage launch
    u_p, work_p, dt_p = u.clone(), f.new_work(), dt.clone()
    f.profile_enable(True)
    f.run(u_p, work_p, dt_p, steps, w.cfl)
    torch.cuda.synchronize()
    f.profile_enable(False)
    eager_ms, eager_launches = f.profile_read()
    del u_p, work_p, dt_p
    bad = f.check_state(u, work)
    if bad:
        print(f"non-physical state after the timed steps ({bad} cells)", file=sys.stderr)
        sys.exit(3)
    tot = f.conserved_totals(u, work).cpu().numpy()
    return {"f": f, "u": u.cpu().numpy(), "totals": tot, "elapsed": elapsed,
            "avg_launch_s": graph_ms / 1e3 / (3 * steps), "launches": 3 * steps,
            "eager_avg_launch_s": eager_ms / 1e3 / max(eager_launches, 1)}


def roofline_sweep(steps: int) -> dict:
    """The stage kernels on forests far larger than the last-level cache:
    2-D 128 x 128 roots of 16 x 16 cells at degrees 1 and 2, 3-D 16^3 roots of
    8^3 cells at degrees 1 and 2 (FP64), and the 3-D degree-2 forest with the
    FP32 residual, its volume integral on the vector unit and on the matrix
    cores; the 2-D 64 x 64-root degree-2 forest and the 3-D degree-1 forest
    also with a rotated frame on every root and with bilinear / trilinear
    roots.  Per case: the
    average stage-kernel duration (HIP events around every stage launch of
    `steps` eager steps), its algorithmic bytes, the fraction of the HBM
    roof, and the estimated flop rate against the FP64 (or FP32) roof."""
    from paper_2502_12620_amd import dgamr as G
    from paper_2502_12620_amd import workloads as W
    from paper_2502_12620_amd.measure import run_workload

    cases = [(W.roofline_2d(128, 1), G.FP64, 0, "affine"), (W.roofline_2d(128, 2), G.FP64, 0, "affine"),
             (W.roofline_3d(16, 1), G.FP64, 0, "affine"), (W.roofline_3d(16, 2), G.FP64, 0, "affine"),
             (W.roofline_3d(16, 2), G.FP32, 0, "affine"), (W.roofline_3d(16, 2), G.FP32, 1, "affine")]
    # rotated frames on every root, and bilinear / trilinear roots (the stage
    # time spans the guard fill and the stage kernel)
    cases += [(W.roofline_2d(64, 2), G.FP64, 0, rk) for rk in ("affine", "rotated", "mapped")]
    cases += [(W.roofline_3d(16, 1), G.FP64, 0, rk) for rk in ("rotated", "mapped")]
    out = {}
    for w, prec, mf, rk in cases:
        r = run_workload(w, steps, warmup=2, precision=prec, mfma=mf, roots=rk)
        key = w.name + ("_fp32" + ("_mfma" if mf else "") if prec == G.FP32 else "_fp64")
        if rk != "affine" or w.name == "rs_vortex2d_k64_p2":
            key += "_" + rk
        # (the flop estimate is that of the affine kernels: left out for
        # the other root kinds)
        keep = ("leaves", "dofs", "state_MB", "stage_kernel_us", "algorithmic_bytes_per_dof", "achieved_GBs",
                "hbm_frac", "mfma_volume", "dof_stage_per_s") + (
                    ("est_TFLOPs", "fp64_frac", "fp32_frac") if rk == "affine" else ("roots",))
        out[key] = {k: r[k] for k in keep if k in r}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--hanging", choices=["paper", "conservative"], default="paper")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-legs", action="store_true", help="time the oracle on the benchmark workload only")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-residual run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 512-forest run")
    ap.add_argument("--batched-repeats", type=int, default=10)
    ap.add_argument("--no-sweep", action="store_true", help="skip the large-forest stage-kernel roofline runs")
    ap.add_argument("--sweep-steps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the whole forest lives on one "
              "MI355X; sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_12620_amd import dgamr as G
    from paper_2502_12620_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.vortex_c2()
    hang = G.HANG_PAPER if args.hanging == "paper" else G.HANG_CONSERVATIVE
    r64 = time_path(G, w, G.FP64, hang, args.steps, args.warmup)
    n = r64["f"].n_leaves
    ab = algorithmic_bytes_per_stage(w, n)
    dof = ab["dof"]
    r32 = time_path(G, w, G.FP32, hang, args.steps, args.warmup) if not args.no_fp32 else None
    sweep = roofline_sweep(args.sweep_steps) if not args.no_sweep else None

    value = dof * 3 * args.steps / r64["elapsed"]
    avg_s = r64["avg_launch_s"]
    achieved = ab["bytes_per_launch"] / avg_s / 1e9
    traffic = read_counter_traffic(w.name)
    out = {
        "metric": "DOF-stage updates/s",
        "value": value,
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "leaves": n, "cells": n * w.n_cell ** w.dim, "dofs": dof,
                   "degree": w.degree, "n_cell": w.n_cell, "hanging": args.hanging, "precision": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage2v (fused residual + RK stage, one lane per cell and variable)",
                     "avg_launch_us": avg_s * 1e6, "launches": r64["launches"],
                     "timing": "HIP events around the timed graph launch / stage launches in it",
                     "eager_avg_launch_us": r64["eager_avg_launch_s"] * 1e6,
                     "algorithmic_bytes_per_launch": ab["bytes_per_launch"],
                     "algorithmic_bytes_per_dof": ab["bytes_per_dof"]},
    }
    if sweep is not None:
        out["roofline_sweep"] = sweep
    if r32 is not None:
        out["fp32_residual"] = {
            "value": dof * 3 * args.steps / r32["elapsed"], "unit": "DOF-stage updates/s",
            "ms_per_step": r32["elapsed"] / args.steps * 1e3, "dtype": "f32 residual, f64 state",
            "kernel": "k_stage<float> (fused residual + RK stage, one thread per cell)",
            "avg_launch_us": r32["avg_launch_s"] * 1e6,
            "achieved_GBs": ab["bytes_per_launch"] / r32["avg_launch_s"] / 1e9}
    if not args.no_batched:
        from paper_2502_12620_amd.measure import batched_run

        b = batched_run(512, args.batched_repeats)
        out["batched"] = {k: b[k] for k in ("workload", "forests", "leaves", "dofs", "steps_per_batch", "repeats",
                                            "batch_wall_s_p50", "batch_wall_s_p99", "dof_stage_per_s",
                                            "sequential_dof_stage_per_s", "speedup_vs_sequential",
                                            "max_rel_diff_vs_plain_path", "pools", "concurrent_branches",
                                            "launches_per_step", "stage_launches_per_stage", "launch_note",
                                            "per_pool", "batch_achieved_GBs", "batch_hbm_frac")}
    if not args.no_cpu:
        cpu, u_ref, tot_ref, tot0 = cpu_baseline(w, args.warmup + args.steps, args.cpu_budget,
                                                 legs=not args.no_cpu_legs)
        out["cpu_baseline"] = cpu
        out["accuracy_vs_oracle"] = {"steps": args.warmup + args.steps,
                                     "fp64": accuracy(r64["u"], r64["totals"], u_ref, tot_ref, tot0)}
        if r32 is not None:
            out["accuracy_vs_oracle"]["fp32_residual"] = accuracy(r32["u"], r32["totals"], u_ref, tot_ref, tot0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
