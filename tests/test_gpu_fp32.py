"""GPU parity of the FP32 residual path (precision FP32): residual
arithmetic in FP32, state, stage combination, limiter and totals in FP64.

Tolerances.  The residual of one cell is a signed sum of at most
n_t = d*N_q + 2d*N_f products of table entries and fluxes, each term rounded
at most a few times, so |R32 - R64| <= c * n_t * u32 * S with u32 = 2^-24
and S the largest term (about max|F| * 2/h * max table entry); on the
vortex data S is within a factor 10 of max|R|.  That gives a per-variable
relative bound of about 5e-5 at p = 3 in 3-D; the tests use 1e-4 for the
residual.  The state after n stages differs by about n * dt * |dR|, far
below the residual's relative error; the 2-D AMR vortex workload's bar is
density L2(U32 - U_orc) / L2(U_orc) <= 1e-5 after its 200 steps."""
import numpy as np
import pytest

import oracle as O
from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import make_pair, rel_diff, small_c2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_RES32 = 1e-4
TOL_L2_C2 = 1e-5


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _l2_rel(got, ref, v=0):
    return float(np.linalg.norm(got[:, v] - ref[:, v]) / np.linalg.norm(ref[:, v]))


def _forest(dim, p, N, levels, bc=0):
    roots = (2, 2) if dim == 2 else (2, 2, 1)
    hi = (2.0, 2.0) if dim == 2 else (2.0, 2.0, 1.0)
    w = W.Workload(f"t{dim}{p}", dim, p, N, roots, (0.0,) * dim, hi, (bc,) * dim, levels, W.IC_VORTEX,
                   [3.0, 1.0, 1.0, 0.5, 0.3, 2.0, 2.0], 1)
    rules = []
    if levels >= 2:
        rules.append(lambda w_, keys: np.array([1 if k[0] == 0 else 0 for k in keys], np.int8))
    if levels >= 3:
        rules.append(lambda w_, keys: np.array([1 if (k[0] == 0 and k[2] == 1 and k[3] == 1) else 0
                                                for k in keys], np.int8))
    w.initial_refinement = rules
    return w


def _physical_state(orc, w, seed):
    rng = np.random.default_rng(seed)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    u[:, :, 1:, :] += 0.01 * rng.standard_normal(u[:, :, 1:, :].shape)
    return u


CASES32 = [(2, 1, 6, 3), (2, 2, 16, 2), (2, 3, 10, 3), (3, 1, 4, 3), (3, 2, 6, 2), (3, 3, 4, 2)]


@pytest.mark.parametrize("dim,p,N,levels", CASES32)
@pytest.mark.parametrize("hanging", [0, 1])
def test_fp32_residual_against_the_oracle(dim, p, N, levels, hanging):
    G = _G()
    w = _forest(dim, p, N, levels)
    orc, gpu = make_pair(w, hanging=hanging, precision=G.FP32)
    u = _physical_state(orc, w, seed=dim * 100 + p * 10 + N)
    r_ref = orc.residual(u)
    ud = _cuda(u)
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    rd = gpu.new_residual()
    assert rd.dtype == torch.float32
    gpu.dg_residual(ud, gd, rd)
    err = rel_diff(_host(rd).astype(np.float64), r_ref)
    print(f"fp32 residual d={dim} p={p} N={N} levels={levels} hanging={hanging}: rel err {err.max():.3e}")
    assert err.max() <= TOL_RES32
    # FP32 is not the FP64 answer rounded once: it must differ at the FP32
    # level somewhere, which shows the FP32 kernel ran
    assert err.max() > 1e-9


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 2)])
def test_fp32_fused_step_matches_the_entry_points(dim, p):
    """step() (fused FP32 stage kernels) against fill + dg_residual (FP32 r)
    + rk_stage per stage; both FP32, so equal to FP32 rounding."""
    G = _G()
    w = _forest(dim, p, 6 if dim == 2 else 4, 3)
    orc, gpu = make_pair(w, hanging=1, precision=G.FP32)
    u = _physical_state(orc, w, seed=3)
    ud = _cuda(u)
    work = gpu.new_work()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    gpu.compute_dt(0.1, ud, dt, work)
    un, us = ud.clone(), ud.clone()
    g, r = gpu.new_guard(), gpu.new_residual()
    for s in range(3):
        gpu.fill_guardcells(us, g)
        gpu.dg_residual(us, g, r)
        nxt = torch.empty_like(us)
        gpu.rk_stage(s, dt, un, us, r, nxt)
        us = nxt
    fused = ud.clone()
    gpu.step(fused, work, dt, cfl=0.0)
    err = rel_diff(_host(fused), _host(us)).max()
    print(f"fp32 fused vs unfused d={dim} p={p}: {err:.3e}")
    assert err <= 1e-6
    orc.step(u, 0.1)
    err_o = rel_diff(_host(fused), u).max()
    print(f"fp32 step vs oracle d={dim} p={p}: {err_o:.3e}")
    assert err_o <= 1e-5


@pytest.mark.parametrize("hanging", [0, 1])
def test_fp32_c2_full_size_200_steps(hanging):
    """The 2-D two-level AMR vortex workload at full size: 200 SSP-RK3 steps
    with FP32 residuals against the FP64 oracle."""
    G = _G()
    w = W.vortex_c2()
    orc, gpu = make_pair(w, hanging=hanging, precision=G.FP32)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = orc.totals(u)
    for _ in range(w.steps):
        orc.step(u, w.cfl)
    gpu.run(ud, work, dt, w.steps, w.cfl)
    got = _host(ud)
    l2 = [_l2_rel(got, u, v) for v in range(4)]
    drift = np.abs(_host(gpu.conserved_totals(ud, work)) - t0) / np.abs(t0).clip(1e-300)
    print(f"fp32 C2 200 steps hanging={hanging}: rel L2 per variable {l2}, rel mass drift {drift}")
    assert l2[0] <= TOL_L2_C2
    assert max(l2) <= 10 * TOL_L2_C2


def test_fp32_conservative_mode_conserves():
    """In conservative hanging-face mode both sides of every face lift the
    same FP32 flux, so the FP64 totals move only by the FP32 rounding of the
    cell-mean updates."""
    G = _G()
    w = small_c2(4)
    orc, gpu = make_pair(w, hanging=1, precision=G.FP32)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = orc.totals(u)
    gpu.run(ud, work, dt, 100, w.cfl)
    drift = np.abs(_host(gpu.conserved_totals(ud, work)) - t0)
    print(f"fp32 conservative drift after 100 steps: {drift / np.abs(t0)}")
    assert np.all(drift <= 1e-6 * np.abs(t0))


def test_fp32_free_stream_across_refinement():
    G = _G()
    w = _forest(2, 2, 8, 3)
    orc, gpu = make_pair(w, hanging=0, precision=G.FP32)
    ud = gpu.project_ic(W.IC_UNIFORM, [1.0, 0.3, -0.2, 0.0, 1.0])
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    u0 = _host(ud)
    gpu.run(ud, work, dt, 20, 0.1)
    assert rel_diff(_host(ud), u0).max() <= 1e-6


def test_fp32_sedov_3d_with_limiter_and_regrid():
    """The 3-D blast workload (4^3-cell blocks so the oracle finishes in
    seconds) with FP32 residuals, positivity limiter and regrid."""
    G = _G()
    w = W.sedov_c3()
    w.n_cell = 4
    orc, gpu = make_pair(w, limiter=True, precision=G.FP32)
    u = orc.project_ic(O.IC_SEDOV, w.ic_params)
    ud = gpu.project_ic(W.IC_SEDOV, w.ic_params)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for step in range(12):
        if step and step % 6 == 0:
            eta_r = orc.indicator(u)
            flags = np.where(eta_r > w.refine_above, 1, np.where(eta_r < w.coarsen_below, -1, 0)).astype(np.int8)
            u = orc.adapt(flags, u)
            ud = gpu.adapt(flags, ud)
            work = gpu.new_work()
        orc.step(u, w.cfl, limiter=True)
        gpu.step(ud, work, dt, w.cfl)
    got = _host(ud)
    l2 = [_l2_rel(got, u, v) for v in range(5) if np.linalg.norm(u[:, v]) > 0]
    print(f"fp32 Sedov 12 steps: rel L2 per variable {l2}")
    assert max(l2) <= 1e-4
    assert gpu.check_state(ud, work) == 0
