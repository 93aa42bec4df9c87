"""GPU parity: every C-ABI entry point of the HIP library against the oracle
on the same seeded inputs, element by element, plus whole runs of the
workloads.  FP64 bar: 1e-12 relative per variable (max |gpu - oracle| /
max |oracle|); guard cells (pure copies and small mat-vecs) 1e-13 absolute
on O(1) data."""
import numpy as np
import pytest

import oracle as O
from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import make_pair, rel_diff, small_c2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _hip():
    from paper_2502_12620_amd import dgamr as G

    return G


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _forest(dim, p, N, levels, hanging=0, bc=0):
    """A periodic (or outflow) forest with a hanging region: root 0 refined,
    then (levels 3) its first child refined again."""
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


CASES = [(2, 0, 4, 3), (2, 1, 6, 3), (2, 2, 16, 2), (2, 2, 4, 3), (2, 3, 10, 3),
         (3, 0, 4, 2), (3, 1, 4, 3), (3, 2, 6, 2), (3, 3, 4, 2)]


@pytest.mark.parametrize("dim,p,N,levels", CASES)
@pytest.mark.parametrize("hanging", [0, 1])
def test_fill_and_residual_parity(dim, p, N, levels, hanging):
    w = _forest(dim, p, N, levels)
    orc, gpu = make_pair(w, hanging=hanging)
    u = _physical_state(orc, w, seed=dim * 100 + p * 10 + N)
    g_ref = orc.fill_guards(u)
    r_ref = orc.residual(u, g_ref)
    ud = _cuda(u)
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    g = _host(gd)
    assert np.abs(g - g_ref).max() <= 1e-13 * max(1.0, np.abs(g_ref).max())
    rd = gpu.new_residual()
    gpu.dg_residual(ud, gd, rd)
    assert rel_diff(_host(rd), r_ref).max() <= TOL


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 1)])
def test_outflow_faces(dim, p):
    w = _forest(dim, p, 4, 2, bc=W.OUTFLOW)
    orc, gpu = make_pair(w)
    u = _physical_state(orc, w, seed=5)
    ud = _cuda(u)
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    assert np.abs(_host(gd) - orc.fill_guards(u)).max() <= 1e-13 * np.abs(u).max()
    rd = gpu.new_residual()
    gpu.dg_residual(ud, gd, rd)
    assert rel_diff(_host(rd), orc.residual(u)).max() <= TOL


def test_single_root_is_its_own_periodic_neighbour():
    w = W.Workload("one", 2, 2, 8, (1, 1), (0.0, 0.0), (10.0, 10.0), (0, 0), 1, W.IC_VORTEX,
                   [5.0, 5.0, 5.0, 1.0, 1.0, 10.0, 10.0], 3)
    orc, gpu = make_pair(w)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
    assert rel_diff(_host(ud), u).max() <= TOL


def test_rk_stage_dt_totals_parity():
    w = _forest(2, 2, 8, 2)
    orc, gpu = make_pair(w)
    u = _physical_state(orc, w, seed=1)
    r = orc.residual(u)
    ud, rd = _cuda(u), _cuda(r)
    work = gpu.new_work()
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    gpu.compute_dt(0.1, ud, dtd, work)
    dt = orc.dt(u, 0.1)
    assert abs(_host(dtd)[0] - dt) <= 1e-15 * dt
    us = ud + 0.001
    for stage in range(3):
        out = torch.empty_like(ud)
        gpu.rk_stage(stage, dtd, ud, us, rd, out)
        ref = O.rk_combine(stage, dt, u, u + 0.001, r)
        assert rel_diff(_host(out), ref).max() <= TOL
    tot = _host(gpu.conserved_totals(ud, work))
    np.testing.assert_allclose(tot, orc.totals(u), rtol=1e-14)


@pytest.mark.parametrize("dim,p,kind", [(2, 1, O.IC_VORTEX), (2, 3, O.IC_XWAVE), (3, 2, O.IC_SEDOV),
                                        (3, 1, O.IC_UNIFORM)])
def test_project_ic_parity(dim, p, kind):
    w = _forest(dim, p, 4, 2)
    orc, gpu = make_pair(w)
    prm = {O.IC_VORTEX: w.ic_params, O.IC_XWAVE: [0.2, 0.7, 2.0],
           O.IC_SEDOV: [1e-5, 1e3, 1.0, 1.0, 0.5], O.IC_UNIFORM: [1.2, 0.3, -0.2, 0.1, 0.9]}[kind]
    ref = orc.project_ic(kind, prm)
    got = _host(gpu.project_ic(kind, prm))
    assert rel_diff(got, ref).max() <= TOL


def test_limiter_and_indicator_parity():
    w = _forest(3, 2, 4, 2, bc=W.OUTFLOW)
    orc, gpu = make_pair(w)
    rng = np.random.default_rng(4)
    u = orc.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1e-3])
    u[:, :, 1:, :] += 0.05 * rng.standard_normal(u[:, :, 1:, :].shape)  # drives p and rho negative in places
    u[:, 0, 0, :] *= 1.0 + 0.3 * rng.random(u[:, 0, 0, :].shape)
    ud = _cuda(u)
    work = gpu.new_work()
    eta = _host(gpu.indicator(ud, work))
    np.testing.assert_allclose(eta, orc.indicator(u), rtol=1e-15)
    gpu.limit_positivity(ud)
    ref = orc.limit(u.copy())
    assert rel_diff(_host(ud), ref).max() <= TOL


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 1)])
def test_refinement_parity(dim, p):
    w = _forest(dim, p, 4, 3)
    orc, gpu = make_pair(w)
    u = _physical_state(orc, w, seed=2)
    ud = _cuda(u)
    rng = np.random.default_rng(6)
    for _ in range(3):
        flags = rng.integers(-1, 2, size=orc.n_leaves).astype(np.int8)
        u = orc.adapt(flags, u)
        ud = gpu.adapt(flags, ud)
        assert np.array_equal(orc.keys(), gpu.keys())
        assert rel_diff(_host(ud), u).max() <= 1e-14


def test_c1_vortex_20_steps():
    w = W.vortex_c1()
    orc, gpu = make_pair(w)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(w.steps):
        dref = orc.step(u, w.cfl)
        gpu.step(ud, work, dt, w.cfl)
        assert abs(_host(dt)[0] - dref) <= 1e-14 * dref
    assert rel_diff(_host(ud), u).max() <= TOL


@pytest.mark.parametrize("hanging", [0, 1])
def test_c2_full_size_steps(hanging):
    w = W.vortex_c2()
    orc, gpu = make_pair(w, hanging=hanging)
    assert orc.n_leaves == 100
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(5):
        orc.step(u, w.cfl)
        gpu.step(ud, work, dt, w.cfl)
    assert rel_diff(_host(ud), u).max() <= TOL


@pytest.mark.parametrize("hanging", [0, 1])
def test_c2_shape_200_steps(hanging):
    w = small_c2(4)
    orc, gpu = make_pair(w, hanging=hanging)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = orc.totals(u)
    for _ in range(200):
        orc.step(u, w.cfl)
        gpu.step(ud, work, dt, w.cfl)
    assert rel_diff(_host(ud), u).max() <= TOL
    drift = np.abs(_host(gpu.conserved_totals(ud, work)) - t0)
    if hanging == 1:
        assert np.all(drift <= 1e-14 * 200 * np.abs(t0) + 1e-12)


@pytest.mark.parametrize("hanging", [0, 1])
def test_run_folds_the_cfl_step_into_the_stages(hanging):
    w = small_c2(8)
    orc, gpu = make_pair(w, hanging=hanging)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    ud, ud2 = _cuda(u), _cuda(u)
    work, dt, dt2 = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda"), \
        torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(15):
        dref = orc.step(u, w.cfl)
        gpu.step(ud, work, dt, w.cfl)
    gpu.run(ud2, work, dt2, 15, w.cfl)
    assert rel_diff(_host(ud2), _host(ud)).max() <= 1e-14
    assert abs(_host(dt2)[0] - dref) <= 1e-14 * dref
    assert rel_diff(_host(ud2), u).max() <= TOL


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("hanging", [0, 1])
@pytest.mark.parametrize("N", [6, 8, 16])
def test_2d_stage_variants_agree_with_the_oracle(p, hanging, N):
    """Both 2-D stage kernels (one lane per cell and variable; one thread per
    cell) on a three-level forest with ragged and full-size N, against the
    oracle."""
    G = _hip()
    w = _forest(2, p, N, 3)
    orc, gpu = make_pair(w, hanging=hanging)
    u = _physical_state(orc, w, seed=20 + p)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    outs = []
    for variant in (0, 1):
        gpu.set_tuning(G.TUNE_STAGE_VARIANT, variant)
        ud = _cuda(u)
        for _ in range(3):
            gpu.step(ud, work, dt, 0.1)
        outs.append(_host(ud))
    for _ in range(3):
        orc.step(u, 0.1)
    for o in outs:
        assert rel_diff(o, u).max() <= TOL


def test_fused_step_matches_unfused_entry_points():
    w = _forest(2, 2, 8, 3, hanging=0)
    orc, gpu = make_pair(w, hanging=1)
    u = _physical_state(orc, w, seed=3)
    ud = _cuda(u)
    work = gpu.new_work()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    gpu.compute_dt(0.1, ud, dt, work)
    # unfused: fill + residual + rk per stage
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
    assert rel_diff(_host(fused), _host(us)).max() <= 1e-14
    orc.step(u, 0.1)
    assert rel_diff(_host(fused), u).max() <= TOL


def test_sedov_3d_with_limiter_and_regrid():
    """The blast workload's forest (176 leaves) at 4^3-cell blocks, limiter on,
    regrids after steps 4 and 8 by the workload's thresholds."""
    w = W.sedov_c3()
    w.n_cell = 4  # the same forest with 4^3-cell blocks, for an oracle run of seconds
    orc, gpu = make_pair(w, limiter=True)
    assert orc.n_leaves == 176
    u = orc.project_ic(O.IC_SEDOV, w.ic_params)
    ud = gpu.project_ic(W.IC_SEDOV, w.ic_params)
    assert rel_diff(_host(ud), u).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for step in range(12):
        if step in (4, 8):
            eta_r = orc.indicator(u)
            eta_g = _host(gpu.indicator(ud, work))
            np.testing.assert_allclose(eta_g, eta_r, rtol=1e-12)
            flags = np.where(eta_r > w.refine_above, 1, np.where(eta_r < w.coarsen_below, -1, 0)).astype(np.int8)
            u = orc.adapt(flags, u)
            ud = gpu.adapt(flags, ud)
            work = gpu.new_work()
            assert np.array_equal(orc.keys(), gpu.keys())
        orc.step(u, w.cfl, limiter=True)
        gpu.step(ud, work, dt, w.cfl)
    assert rel_diff(_host(ud), u).max() <= TOL
    assert gpu.check_state(ud, work) == 0


@pytest.mark.parametrize("n_cell", [2, 4])
def test_sedov_3d_regrid_changes_the_forest(n_cell):
    """The blast from a forest refined only to level 2 around the centre:
    the regrid after step 3 (thresholds lowered so that the third step's
    density ratio triggers it) refines the centre to level 3, so the
    inheritance, the new links and the hanging faces it creates all run on
    both sides; FP64 parity at 1e-12 with the limiter on."""
    w = W.sedov_c3()
    w.n_cell = n_cell
    w.initial_refinement = w.initial_refinement[:1]
    orc, gpu = make_pair(w, limiter=True)
    assert orc.n_leaves == 120
    u = orc.project_ic(O.IC_SEDOV, w.ic_params)
    ud = gpu.project_ic(W.IC_SEDOV, w.ic_params)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for step in range(7):
        if step == 3:
            eta_r = orc.indicator(u)
            np.testing.assert_allclose(_host(gpu.indicator(ud, work)), eta_r, rtol=1e-12)
            flags = np.where(eta_r > 1.01, 1, np.where(eta_r < 1.001, -1, 0)).astype(np.int8)
            u = orc.adapt(flags, u)
            ud = gpu.adapt(flags, ud)
            work = gpu.new_work()
            assert orc.n_leaves > 120 and np.array_equal(orc.keys(), gpu.keys())
        dref = orc.step(u, w.cfl, limiter=True)
        gpu.step(ud, work, dt, w.cfl)
        assert abs(_host(dt)[0] - dref) <= 1e-13 * dref
    assert rel_diff(_host(ud), u).max() <= TOL


def test_stale_buffers_are_rejected_after_a_refinement():
    """After a refinement grows the forest, a state or work buffer sized for
    the old forest is refused by the binding before any kernel runs."""
    w = _forest(2, 1, 4, 2)
    orc, gpu = make_pair(w)
    ud = gpu.project_ic(W.IC_VORTEX, w.ic_params)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    flags = np.zeros(gpu.n_leaves, np.int8)
    flags[-1] = 1
    ud2 = gpu.adapt(flags, ud)
    with pytest.raises(ValueError, match="work"):
        gpu.step(ud2, work, dt)
    with pytest.raises(ValueError, match="u"):
        gpu.step(ud, gpu.new_work(), dt)
    with pytest.raises(ValueError, match="dtype"):
        gpu.step(ud2.float(), gpu.new_work(), dt)
    gpu.step(ud2, gpu.new_work(), dt)  # the right sizes run


def test_nonphysical_state_is_reported():
    w = _forest(2, 1, 4, 1)
    orc, gpu = make_pair(w)
    u = orc.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1.0])
    u[0, 3, 0, 5] = -1.0  # negative energy planted on the host
    ud = _cuda(u)
    assert gpu.check_state(ud, gpu.new_work()) == 1


def test_sedov_full_size_steps():
    """The 3-D blast workload at full size (176 leaves of 8^3 cells, degree 2,
    limiter) for 3 steps against the oracle."""
    w = W.sedov_c3()
    orc, gpu = make_pair(w, limiter=True)
    assert orc.n_leaves == 176
    u = orc.project_ic(O.IC_SEDOV, w.ic_params)
    ud = gpu.project_ic(W.IC_SEDOV, w.ic_params)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, w.cfl, limiter=True)
        gpu.step(ud, work, dt, w.cfl)
        assert abs(_host(dt)[0] - dref) <= 1e-13 * dref
    assert rel_diff(_host(ud), u).max() <= TOL
