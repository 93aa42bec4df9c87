"""Measurement helpers for an MI355X (not part of the solver path).

    python -m paper_2502_12620_amd.measure copy  [--mb 1024]
        a plain device-to-device copy of known size, the calibration kernel
        for the FETCH_SIZE / WRITE_SIZE counters;
    python -m paper_2502_12620_amd.measure sweep [--steps 10]
        the roofline sweep: uniform 2-D and 3-D vortex forests large enough
        to live in HBM (above the 256 MB last-level cache), FP64 stage kernel
        timed with HIP events around each launch;
    python -m paper_2502_12620_amd.measure batch [--forests 512]
        the batched workload: independent 2-D forests in one pool per degree,
        autotuned, one HIP graph per batch of steps; batch wall time p50/p99
        and DOF-stage/s against the same forests solved one after another;
    python -m paper_2502_12620_amd.measure convection [--dim 2 --degree 2 --n-cell 8]
        the scalar convection workload (Sec. 5.1) with indicator-driven
        regrids to t_end: DOF-stage/s and the L2 distance to the projected
        exact solution;
    python -m paper_2502_12620_amd.measure diffusion [--degree 2]
        the diffusion workload (Sec. 5.2) with indicator-driven regrids to
        t = 0.2: DOF-stage/s and the L2 distance to the projected exact
        solution;
    python -m paper_2502_12620_amd.measure sedov
        the 3-D blast workload end to end (limiter, regrid every 10 steps)
        with FP64 and with FP32 residuals, and their L1 / L2 difference;
    python -m paper_2502_12620_amd.measure serve [--requests 40 --rates 200]
        the served workload: a Poisson stream of 2-D/3-D solves through the
        continuous-batching request loop, at one or more arrival rates;
        latency p50/p99 and DOF-stage/s against plain sequential solves of
        the same requests.

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
FP32_PEAK_TFLOPS = 157.3  # dense FP32 on the matrix cores (and the vector unit's FMA rate)
# estimated FP64 flops per DOF per stage (volume evaluate + flux + project,
# face traces + Rusanov + lift), by (dim, degree)
FLOP_PER_DOF = {(2, 1): 76, (2, 2): 120, (2, 3): 176, (3, 1): 207, (3, 2): 480, (3, 3): 945}


def stage_bytes_per_dof(dim: int, n_cell: int, stage=None) -> float:
    """Algorithmic bytes of the fused stage kernel per DOF: U_s read, U_n
    read on stages 2-3, U_next write, face layer of the neighbours; for one
    stage (0, 1, 2) or averaged over the three."""
    face = 8.0 * 2 * dim / n_cell
    per = [16.0, 24.0, 24.0]
    return (sum(per) / 3.0 if stage is None else per[stage]) + face


def run_workload(w, steps: int, warmup: int = 3, precision=G.FP64, variant=-1, rows=0, mfma=0, roots="affine"):
    """Time w's steps; roots "mapped" moves the root grid nodes smoothly
    (bilinear / trilinear roots), "rotated" gives every root a seeded
    frame.  The stage time is that of each stage's launches; the
    algorithmic bytes are the same for every kind of root."""
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma, precision=precision)
    f.set_tuning(G.TUNE_STAGE_VARIANT, variant)
    f.set_tuning(G.TUNE_SLAB_ROWS, rows)
    f.set_tuning(G.TUNE_MFMA, mfma)
    if roots == "mapped":
        f.set_root_nodes(W.smooth_root_nodes(w))
    elif roots == "rotated":
        f.set_root_frames(W.random_root_frames(w))
    elif roots != "affine":
        raise ValueError(f"unknown root kind {roots}")
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
    fp32 = precision == G.FP32
    out = {"workload": w.name, "roots": roots, "precision": "fp32" if fp32 else "fp64", "variant": variant,
            "rows": rows, "mfma_volume": bool(mfma and fp32 and mfma_volume(w.dim, w.degree)),
            "dim": w.dim, "degree": w.degree, "leaves": n, "dofs": dof,
            "state_MB": dof * 8 / 1e6, "steps": steps, "dof_stage_per_s": dof * 3 * steps / el,
            "stage_kernel_us": avg * 1e6, "algorithmic_bytes_per_dof": bpd, "achieved_GBs": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "est_TFLOPs": flops,
            "nonphysical_cells": bad}
    if fp32:
        out["fp32_frac"] = flops / FP32_PEAK_TFLOPS
    else:
        out["fp64_frac"] = flops / FP64_PEAK_TFLOPS
    return out


def mfma_volume(dim: int, degree: int) -> bool:
    """Whether the FP32 stage kernel's volume integral runs on the matrix
    cores (degree >= 2, except 3-D degree 3)."""
    return degree >= 2 and not (dim == 3 and degree == 3)


def cmd_sweep(args):
    cases = [W.roofline_2d(k, p) for k in (32, 64, 128) for p in (1, 2)]
    cases += [W.roofline_2d(64, 3)]
    cases += [W.roofline_3d(16, p) for p in (1, 2)] + [W.roofline_3d(8, 3)]
    for w in cases:
        if args.only and w.name not in args.only.split(","):
            continue
        prec = G.FP32 if args.precision == "fp32" else G.FP64
        variants = [0, 1] if (args.variants and prec == G.FP64) else [-1]
        for var in variants:
            for rows in [int(r) for r in args.rows.split(",")]:
                for mf in [int(m) for m in args.mfma.split(",")]:
                    for rk in args.roots.split(","):
                        print(json.dumps(run_workload(w, args.steps, precision=prec, variant=var, rows=rows,
                                                      mfma=mf, roots=rk)), flush=True)


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
    out = {"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "ms": ms,
           "GBs_read_plus_write": 2 * n * 8 / ms / 1e6}
    if args.triad:
        # the traffic of an RK stage 2 or 3 (two arrays read, one written)
        # through torch's elementwise kernel
        third = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, dst, alpha=0.25, out=third)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.reps):
            torch.add(src, dst, alpha=0.25, out=third)
        e1.record()
        torch.cuda.synchronize()
        tms = e0.elapsed_time(e1) / args.reps
        out.update({"triad_ms": tms, "triad_GBs": 3 * n * 8 / tms / 1e6})
    print(json.dumps(out), flush=True)


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def _forest(w, precision=G.FP64):
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma, precision=precision)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    return f


def cmd_batch(args):
    print(json.dumps(batched_run(args.forests, args.repeats, args.precision)), flush=True)


def batched_run(forests: int = 512, repeats: int = 20, precision: str = "fp64") -> dict:
    """The batched workload: pools per degree, autotuned, one HIP graph of a
    batch (20 steps of every forest); batch wall times over `repeats`
    replays, and the same forests solved one after another (dgamr_run)."""
    ws = W.batched_forests(forests, seed=2502)
    steps = ws[0].steps
    prec = G.FP32 if precision == "fp32" else G.FP64
    groups = {}
    for w in ws:
        groups.setdefault(w.degree, []).append((w, _forest(w, prec)))
    pools, members = [], []
    t_setup = time.perf_counter()
    for p in sorted(groups):
        lst = groups[p]
        pool = G.Pool(2, p, 16, sum(f.n_leaves for _, f in lst), len(lst), precision=prec)
        for w, f in lst:
            mid, first = pool.admit(f, w.cfl)
            f.project_ic(G.IC_VORTEX, w.ic_params, u=pool.view(first, f.n_leaves))
            members.append((w, f, pool, first))
        pools.append(pool)
    torch.cuda.synchronize()
    tune = [pool.autotune() for pool in pools]
    # the autotuner left the arenas untouched; restart from the initial state
    graph = G.Graph(pools, nsteps=steps)
    setup_s = time.perf_counter() - t_setup
    dofs = sum(w.dofs(f.n_leaves) for w, f in ((w, f) for w, f, _, _ in members))
    leaves = sum(f.n_leaves for _, f, _, _ in members)
    # one replay from the initial state: results against the plain path
    graph.launch()
    torch.cuda.synchronize()
    # plain FP64 path: every forest alone, one after another (dgamr_run)
    seq_times, max_rel = [], 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for w, f, pool, first in members:
        u = f.project_ic(G.IC_VORTEX, w.ic_params)
        work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
        f.run(u, work, dt, 1, w.cfl)  # warm-up of this forest's path
        u = f.project_ic(G.IC_VORTEX, w.ic_params)
        torch.cuda.synchronize()
        e0.record()
        f.run(u, work, dt, steps, w.cfl)
        e1.record()
        torch.cuda.synchronize()
        seq_times.append(e0.elapsed_time(e1) / 1e3)
        got = pool.view(first, f.n_leaves)
        max_rel = max(max_rel, float((got - u).abs().max() / u.abs().max()))
    seq_total = sum(seq_times)
    # timed replays (the state keeps advancing: each replay is `steps` more steps)
    times = []
    for _ in range(repeats):
        e0.record()
        graph.launch()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    med = _pct(times, 50)
    # per degree class: the pool's stage kernel timed alone by the autotuner
    # (its first stage, which does not read U_n), against the HBM roof; and
    # the whole batch's stage traffic over the batch wall time (the pools run
    # on parallel branches of the graph)
    bpd0, bpd = stage_bytes_per_dof(2, 16, stage=0), stage_bytes_per_dof(2, 16)
    per_pool = {}
    for p, (v, r, g, us) in zip(sorted(groups), tune):
        pd = sum(w.dofs(f.n_leaves) for w, f in groups[p])
        gbs = pd * bpd0 / (us * 1e-6) / 1e9
        per_pool[f"p{p}"] = {"forests": len(groups[p]), "dofs": pd, "first_stage_us_alone": us, "achieved_GBs": gbs,
                             "hbm_frac": gbs / HBM_PEAK_GBS}
    batch_gbs = dofs * bpd * 3 * steps / med / 1e9
    out = {"workload": f"batched_{forests}_forests_2d", "forests": len(ws), "leaves": leaves, "dofs": dofs,
           "pools": len(pools), "concurrent_branches": len(pools),
           "launches_per_step": 5 * len(pools),
           "stage_launches_per_stage": len(pools),
           "launch_note": "per pool and step: two CFL reductions and three stage kernels; the pools' launches run "
                          "on parallel branches of one HIP graph",
           "per_pool": per_pool, "batch_achieved_GBs": batch_gbs, "batch_hbm_frac": batch_gbs / HBM_PEAK_GBS,
           "precision": precision, "steps_per_batch": steps, "repeats": repeats,
           "batch_wall_s_p50": med, "batch_wall_s_p99": _pct(times, 99), "batch_wall_s_min": min(times),
           "dof_stage_per_s": dofs * 3 * steps / med,
           "sequential_plain_s": seq_total, "sequential_dof_stage_per_s": dofs * 3 * steps / seq_total,
           "speedup_vs_sequential": seq_total / med,
           "max_rel_diff_vs_plain_path": max_rel,
           "autotune": {f"p{p}": {"variant": v, "rows": r, "grid": g, "stage_us": us}
                        for p, (v, r, g, us) in zip(sorted(groups), tune)},
           "setup_s": setup_s}
    return out


def _sedov_gpu(w, precision):
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma, precision=precision,
                 limiter=G.LIMITER_POSITIVITY)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    u = f.project_ic(G.IC_SEDOV, w.ic_params)
    work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = f.conserved_totals(u, work).cpu().numpy()
    torch.cuda.synchronize()
    start = time.perf_counter()
    dof_stages, regrid_s = 0, 0.0
    for step in range(w.steps):
        if step and step % w.regrid_every == 0:
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            eta = f.indicator(u, work).cpu().numpy()
            flags = ((eta > w.refine_above).astype("int8") - (eta < w.coarsen_below).astype("int8"))
            u = f.adapt(flags, u)
            work = f.new_work()
            torch.cuda.synchronize()
            regrid_s += time.perf_counter() - r0
        f.step(u, work, dt, w.cfl)
        dof_stages += 3 * w.dofs(f.n_leaves)
    torch.cuda.synchronize()
    el = time.perf_counter() - start
    bad = f.check_state(u, work)
    tot = f.conserved_totals(u, work).cpu().numpy()
    return f, u.cpu().numpy(), {"wall_s": el, "regrid_s": regrid_s, "dof_stage_per_s": dof_stages / el,
                                "final_leaves": f.n_leaves, "nonphysical_cells": bad,
                                "rel_mass_drift": float(abs(tot[0] - t0[0]) / abs(t0[0]))}


def cmd_sedov(args):
    w = W.sedov_c3()
    out = {"workload": w.name, "steps": w.steps}
    res = {}
    for name, prec in (("fp64", G.FP64), ("fp32", G.FP32)):
        f, u, r = _sedov_gpu(w, prec)
        res[name] = (f.keys(), u)
        out[name] = r
    import numpy as np

    (k64, u64), (k32, u32) = res["fp64"], res["fp32"]
    if np.array_equal(k64, k32):
        d = u32[:, 0] - u64[:, 0]
        out["fp32_vs_fp64"] = {"rel_l1_density": float(np.abs(d).sum() / np.abs(u64[:, 0]).sum()),
                               "rel_l2_density": float(np.linalg.norm(d) / np.linalg.norm(u64[:, 0])),
                               "rel_max_all": float(np.abs(u32 - u64).max() / np.abs(u64).max())}
    else:
        out["fp32_vs_fp64"] = "the regrids produced different forests"
    print(json.dumps(out), flush=True)


def _ref_mass(dim, degree):
    """Reference-cell mass of each basis mode, prod_a 2/(2 m_a + 1), graded
    mode order (total degree |m| ascending, then m_x, m_y descending)."""
    out = []
    for s in range(degree + 1):
        for mx in range(s, -1, -1):
            if dim == 2:
                out.append((2 / (2 * mx + 1)) * (2 / (2 * (s - mx) + 1)))
            else:
                for my in range(s - mx, -1, -1):
                    out.append((2 / (2 * mx + 1)) * (2 / (2 * my + 1)) * (2 / (2 * (s - mx - my) + 1)))
    return out


def cmd_convection(args):
    """The scalar convection workload of Sec. 5.1 on the GPU: regrids by the
    block indicator, SSP-RK3 to t_end (last step shortened to land on it),
    DOF-stage/s, and the L2 distance between the solution and the L2
    projection of the exact (translated) solution on the final forest."""
    if args.rotated:
        w = W.convection_2d_rotated(degree=args.degree, n_cell=args.n_cell)
    elif args.distorted:
        w = W.convection_2d_distorted(degree=args.degree, n_cell=args.n_cell)
    elif args.dim == 2:
        w = W.convection_2d(degree=args.degree, n_cell=args.n_cell)
    else:
        w = W.convection_3d(degree=args.degree, n_cell=args.n_cell)
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                 equation=G.EQ_ADVECTION, velocity=w.velocity[:w.dim])
    nodes = getattr(w, "nodes", None)
    if nodes is not None:
        f.set_root_nodes(nodes)
    if getattr(w, "frames", None) is not None:
        f.set_root_frames(w.frames)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    u = f.project_ic(G.IC_COSINE, w.ic_params)
    work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    t, steps, dof_stages, regrids = 0.0, 0, 0, 0
    torch.cuda.synchronize()
    start = time.perf_counter()
    while t < w.t_end - 1e-14:
        if w.regrid_every and steps % w.regrid_every == 0:
            eta = f.indicator(u, work).cpu().numpy()
            flags = W.regrid_flags(w, f.keys(), eta)
            if (flags != 0).any():
                u = f.adapt(flags, u)
                work = f.new_work()
                regrids += 1
        f.compute_dt(w.cfl, u, dt, work)
        h = float(dt.item())
        if t + h > w.t_end:
            dt.fill_(w.t_end - t)
            h = w.t_end - t
        f.step(u, work, dt, cfl=0.0)
        t += h
        steps += 1
        dof_stages += 3 * w.dofs(f.n_leaves)
    torch.cuda.synchronize()
    el = time.perf_counter() - start
    ex = f.project_ic(G.IC_COSINE, w.ic_params, t=w.t_end)
    if nodes is not None:
        l2 = _mapped_l2(f, w, (u - ex).cpu().numpy())
    else:
        vol = torch.tensor([g for g in _leaf_volumes(f, w)], dtype=torch.float64, device="cuda")
        mass = torch.tensor(_ref_mass(w.dim, w.degree), dtype=torch.float64, device="cuda")
        d2 = ((u - ex) ** 2 * mass[None, None, :, None]).sum(dim=(1, 2, 3))
        l2 = float(torch.sqrt((d2 * vol / 2 ** w.dim).sum()))
    out = {"workload": w.name, "degree": w.degree, "n_cell": w.n_cell, "t_end": w.t_end, "steps": steps,
           "regrids": regrids, "final_leaves": f.n_leaves, "wall_s": el, "dof_stage_per_s": dof_stages / el,
           "l2_to_projected_exact": l2}
    print(json.dumps(out), flush=True)


def _mapped_l2(f, w, d):
    """L2 norm over the physical cells of a scalar field given by its
    coefficients d[leaf, 0, mode, cell] on bilinear roots: per cell the
    Gauss rule with p+1 points per axis (exact for the square of a degree-p
    polynomial times the bilinear det J), with the cell corners from the
    root nodes."""
    import numpy as np

    p, N = w.degree, w.n_cell
    x, wq = np.polynomial.legendre.leggauss(p + 1)
    modes = [(mx, s - mx) for s in range(p + 1) for mx in range(s, -1, -1)]
    leg = np.polynomial.legendre.legval
    ph = np.array([[leg(x[i], [0] * a + [1]) * leg(x[j], [0] * b + [1]) for (a, b) in modes]
                   for j in range(p + 1) for i in range(p + 1)])  # (point, mode), x fastest
    ww = np.array([wq[i] * wq[j] for j in range(p + 1) for i in range(p + 1)])
    xi = np.array([(x[i], x[j]) for j in range(p + 1) for i in range(p + 1)])
    nodes = w.nodes
    total = 0.0
    for li, (tree, level, ki, kj, _) in enumerate(f.keys().tolist()):
        rx, ry = tree % w.roots[0], tree // w.roots[0]
        n00, n10, n01, n11 = nodes[ry, rx], nodes[ry, rx + 1], nodes[ry + 1, rx], nodes[ry + 1, rx + 1]
        span = 2 ** (level - 1)
        for c in range(N * N):
            ci, cj = c % N, c // N
            cx = []
            for b in range(4):
                s0 = (ki + (ci + (b & 1)) / N) / span
                s1 = (kj + (cj + (b >> 1)) / N) / span
                cx.append((1 - s0) * (1 - s1) * n00 + s0 * (1 - s1) * n10 + (1 - s0) * s1 * n01 + s0 * s1 * n11)
            cx = np.array(cx)
            e, h = xi[:, 0], xi[:, 1]
            jxe = 0.25 * ((1 - h)[:, None] * (cx[1] - cx[0]) + (1 + h)[:, None] * (cx[3] - cx[2]))
            jxh = 0.25 * ((1 - e)[:, None] * (cx[2] - cx[0]) + (1 + e)[:, None] * (cx[3] - cx[1]))
            det = jxe[:, 0] * jxh[:, 1] - jxh[:, 0] * jxe[:, 1]
            vals = ph @ d[li, 0, :, c]
            total += float((ww * det * vals ** 2).sum())
    return total ** 0.5


def cmd_diffusion(args):
    """The diffusion workload of Sec. 5.2 on the GPU: regrids by the block
    indicator every 10 steps, SSP-RK3 at the diffusive CFL number to
    t_end (the last step shortened to land on it), DOF-stage/s, and the L2
    distance between the solution and the L2 projection of the exact
    solution on the final forest."""
    w = W.diffusion_2d(degree=args.degree)
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                 equation=G.EQ_DIFFUSION, nu=w.nu, exact_a=w.exact_a)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    u = f.project_ic(G.IC_EXP, [])
    f.time = 0.0
    work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    steps, dof_stages, regrids = 0, 0, 0
    torch.cuda.synchronize()
    start = time.perf_counter()
    while f.time < w.t_end - 1e-14:
        if steps % w.regrid_every == 0:
            eta = f.indicator(u, work).cpu().numpy()
            flags = W.regrid_flags(w, f.keys(), eta)
            if (flags != 0).any():
                u = f.adapt(flags, u)
                work = f.new_work()
                regrids += 1
        f.compute_dt(1.0, u, dt, work)  # dt per unit CFL number: dt is proportional to it
        per_cfl = float(dt.item())
        cfl = min(w.cfl, (w.t_end - f.time) / per_cfl)
        f.step(u, work, dt, cfl=cfl)
        steps += 1
        dof_stages += 3 * w.dofs(f.n_leaves)
        if steps % 20000 == 0:
            print(json.dumps({"progress": "diffusion", "steps": steps, "t": f.time}), flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - start
    ex = f.project_ic(G.IC_EXP, [], t=f.time)
    vol = torch.tensor([g for g in _leaf_volumes(f, w)], dtype=torch.float64, device="cuda")
    mass = torch.tensor(_ref_mass(w.dim, w.degree), dtype=torch.float64, device="cuda")
    d2 = ((u - ex) ** 2 * mass[None, None, :, None]).sum(dim=(1, 2, 3))
    l2 = float(torch.sqrt((d2 * vol / 2 ** w.dim).sum()))
    out = {"workload": w.name, "degree": w.degree, "n_cell": w.n_cell, "t_end": f.time, "steps": steps,
           "regrids": regrids, "final_leaves": f.n_leaves, "wall_s": el, "dof_stage_per_s": dof_stages / el,
           "l2_to_projected_exact": l2}
    print(json.dumps(out), flush=True)


def _leaf_volumes(f, w):
    """Cell volume of every leaf, from the keys (level) and the root box."""
    keys = f.keys()
    root = [(w.hi[a] - w.lo[a]) / w.roots[a] for a in range(w.dim)]
    out = []
    for k in keys:
        v = 1.0
        for a in range(w.dim):
            v *= root[a] / 2 ** (int(k[1]) - 1) / w.n_cell
        out.append(v)
    return out


def _sequential_service(reqs):
    """Each request solved alone (plain FP64 path, dgamr_run): its service
    time in seconds, by request id."""
    service = {}
    for r in reqs:
        w = r.workload
        f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma)
        u = f.project_ic(w.ic_kind, w.ic_params)
        work_buf, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.run(u, work_buf, dt, w.steps, w.cfl)
        torch.cuda.synchronize()
        service[r.rid] = time.perf_counter() - t0
        del f, u, work_buf
        if len(service) % 25 == 0:
            print(json.dumps({"progress": "sequential", "done": len(service)}), flush=True)
    return service


def cmd_serve(args):
    """The served stream at each arrival rate: the same requests (seed
    12620; the rate only scales the arrival times), served by the
    continuous-batching loop, against the same requests solved one after
    another in arrival order (queue replayed from measured service times)."""
    from .serve import Request, Server

    rates = [float(x) for x in args.rates.split(",")]
    service = None
    for rate in rates:
        reqs = [Request(i, t, w) for i, (t, w) in enumerate(W.served_requests(args.requests, seed=12620, rate=rate))]
        classes = sorted({(r.workload.dim, r.workload.degree, r.workload.n_cell) for r in reqs})
        srv = Server(classes, hbm_budget=args.budget_gb * 1e9, max_members=256, tune=args.tune)
        total_work = sum(r.workload.dofs(math.prod(r.workload.roots)) * 3 * r.workload.steps for r in reqs)
        print(json.dumps({"progress": "serving", "rate_per_s": rate, "requests": len(reqs),
                          "dof_stage_total": total_work}), flush=True)

        def progress(r):
            n = sum(1 for q in reqs if q.done >= 0)
            if n % 25 == 0 or n == len(reqs):
                print(json.dumps({"progress": "served", "done": n, "t_s": round(r.done, 3)}), flush=True)

        done = srv.run(reqs, on_done=progress)
        lat = [r.done - r.arrival for r in done]
        wait = [r.admitted - r.arrival for r in done]
        work = sum(r.dofs * 3 * r.workload.steps for r in done)
        out = {"workload": f"served_{args.requests}_requests", "requests": len(done), "rate_per_s": rate,
               "offered_dof_stage_per_s": work / max(r.arrival for r in done),
               "hbm_budget_GB": args.budget_gb, "peak_pool_GB": srv.peak_bytes / 1e9, "makespan_s": srv.makespan,
               "steps_enqueued": srv.steps_enqueued, "pool_rebuilds": srv.rebuilds, "members_moved": srv.moved,
               "deferred_admissions": srv.full_waits,
               "latency_s_p50": _pct(lat, 50), "latency_s_p99": _pct(lat, 99),
               "queue_wait_s_p50": _pct(wait, 50), "queue_wait_s_p99": _pct(wait, 99),
               "dof_stage_per_s": work / srv.makespan}
        del srv
        torch.cuda.empty_cache()
        if service is None:
            service = _sequential_service(sorted(done, key=lambda r: r.arrival))
        clock, seq_lat = 0.0, []
        for r in sorted(done, key=lambda r: r.arrival):
            start = max(clock, r.arrival)
            clock = start + service[r.rid]
            seq_lat.append(clock - r.arrival)
        out.update({"sequential_makespan_s": clock, "sequential_latency_s_p50": _pct(seq_lat, 50),
                    "sequential_latency_s_p99": _pct(seq_lat, 99), "sequential_dof_stage_per_s": work / clock})
        print(json.dumps(out), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--steps", type=int, default=10)
    s.add_argument("--only", default="", help="comma-separated workload names")
    s.add_argument("--variants", action="store_true", help="FP64: time both stage kernels (lane per cell and variable; thread per cell)")
    s.add_argument("--precision", choices=["fp64", "fp32"], default="fp64", help="residual arithmetic")
    s.add_argument("--rows", default="0", help="comma-separated slab heights to time (0: the kernel's own)")
    s.add_argument("--mfma", default="0", help="FP32: comma-separated 1 (volume integral on the matrix cores) / 0")
    s.add_argument("--roots", default="affine", help="comma-separated root kinds: affine, mapped (bilinear / trilinear), rotated (frames)")
    c = sub.add_parser("copy")
    c.add_argument("--mb", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    c.add_argument("--triad", action="store_true", help="also time a two-read one-write elementwise kernel")
    b = sub.add_parser("batch")
    b.add_argument("--forests", type=int, default=512)
    b.add_argument("--repeats", type=int, default=20)
    b.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    sub.add_parser("sedov")
    c2 = sub.add_parser("convection")
    c2.add_argument("--dim", type=int, default=2)
    c2.add_argument("--degree", type=int, default=2)
    c2.add_argument("--n-cell", type=int, default=8)
    c2.add_argument("--distorted", action="store_true", help="2-D, the second root set: four distorted roots")
    c2.add_argument("--rotated", action="store_true", help="2-D, four square roots with rotated frames")
    df = sub.add_parser("diffusion")
    df.add_argument("--degree", type=int, default=2)
    v = sub.add_parser("serve")
    v.add_argument("--requests", type=int, default=40)
    v.add_argument("--rates", default="200", help="comma-separated arrival rates (requests/s)")
    v.add_argument("--budget-gb", type=float, default=96.0)
    v.add_argument("--tune", action="store_true")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    {"sweep": cmd_sweep, "copy": cmd_copy, "batch": cmd_batch, "serve": cmd_serve, "sedov": cmd_sedov,
     "convection": cmd_convection, "diffusion": cmd_diffusion}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
