"""The 3-D stage kernel with one lane per (cell, variable), against the
oracle and against the thread-per-cell kernel: three-level forests (two
hanging levels) with periodic and outflow faces at every degree, slabs of
two or more layers and whole-leaf slabs with a ragged last wave, small and
full-size forests, and graph replay.  Forests it does not take (mortar
faces, the limiter, FP32 residuals) run the thread-per-cell kernel
unchanged."""
import numpy as np
import pytest

from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import make_pair, rel_diff, rel_diff_floored
from tests.test_gpu_parity import TOL, _cuda, _forest, _host, _physical_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _steps(gpu, u, variant, steps, cfl=0.1, rows=0):
    G = _G()
    gpu.set_tuning(G.TUNE_STAGE_VARIANT, variant)
    gpu.set_tuning(G.TUNE_SLAB_ROWS, rows)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        gpu.step(ud, work, dt, cfl)
    return _host(ud)


# (degree, N, slab rows): N = 4 auto (two-layer slabs), N = 4 whole leaf
# (64 cells: 6 waves, 8 unused cell slots), N = 2 whole leaf (one wave, 4
# unused slots), N = 6 three-layer slabs (108 cells), N = 8 two-layer slabs
CASES = [(0, 4, 0), (1, 4, 0), (1, 4, 4), (1, 8, 0), (2, 4, 0), (2, 2, 0), (2, 6, 0), (2, 8, 0), (3, 4, 4),
         (3, 6, 0)]


@pytest.mark.parametrize("p,N,rows", CASES)
@pytest.mark.parametrize("bc", [W.PERIODIC, W.OUTFLOW])
def test_3d_lane_kernel_agrees_with_the_oracle(p, N, rows, bc):
    w = _forest(3, p, N, 3, bc=bc)
    orc, gpu = make_pair(w)
    u = _physical_state(orc, w, seed=40 + p + N)
    lane = _steps(gpu, u, 0, 3, rows=rows)
    cell = _steps(gpu, u, 1, 3)
    for _ in range(3):
        orc.step(u, 0.1)
    assert rel_diff(lane, u).max() <= TOL
    assert rel_diff(cell, u).max() <= TOL
    # (floored: a variable that is zero up to rounding compares absolutely)
    assert rel_diff_floored(lane, cell, floor=1e-2).max() <= 1e-13


@pytest.mark.parametrize("case", ["conservative", "limiter", "fp32"])
def test_forests_it_does_not_take_run_the_thread_per_cell_kernel(case):
    """Mortar faces (conservative hanging mode), the positivity limiter and
    FP32 residual arithmetic: the request for the lane kernel falls back to
    the thread-per-cell kernel, bitwise."""
    G = _G()
    w = _forest(3, 1, 4, 2)
    orc, gpu = make_pair(w, hanging=1 if case == "conservative" else 0, limiter=case == "limiter",
                         precision=G.FP32 if case == "fp32" else None)
    u = _physical_state(orc, w, seed=7)
    assert np.array_equal(_steps(gpu, u, 0, 2), _steps(gpu, u, 1, 2))


@pytest.mark.parametrize("p", [1, 2])
def test_full_size_roofline_forest(p):
    """The 16^3-root roofline forests (41.9 M / 104.9 M DOF): two steps of
    the lane kernel against the thread-per-cell kernel, and the discrete
    mass is conserved (periodic)."""
    G = _G()
    w = W.roofline_3d(16, p)
    outs = []
    for variant in (0, 1):
        f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma)
        f.set_tuning(G.TUNE_STAGE_VARIANT, variant)
        u = f.project_ic(w.ic_kind, w.ic_params)
        work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
        m0 = float(_host(f.conserved_totals(u, work))[0])
        for _ in range(2):
            f.step(u, work, dt, w.cfl)
        assert abs(float(_host(f.conserved_totals(u, work))[0]) - m0) <= 1e-12 * abs(m0)
        # a sample of leaves, all variables and modes
        idx = torch.arange(0, f.n_leaves, 97, device="cuda")
        outs.append(_host(u.index_select(0, idx)))
        del u
    # per variable relative to its largest value; the z momentum of the
    # extruded vortex is zero up to rounding, so its scale is floored at
    # 1e-2 of the largest coefficient
    assert rel_diff_floored(outs[0], outs[1], floor=1e-2).max() <= 1e-13


def test_run_capture_replays_with_the_lane_kernel():
    G = _G()
    w = _forest(3, 2, 8, 3)
    orc, gpu = make_pair(w)
    gpu.set_tuning(G.TUNE_STAGE_VARIANT, 0)
    u = _physical_state(orc, w, seed=3)
    u_g, u_e = _cuda(u), _cuda(u)
    work_g, work_e = gpu.new_work(), gpu.new_work()
    dt_g, dt_e = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2))
    graph = gpu.capture_run(u_g, work_g, dt_g, 2, 0.1)
    for rep in range(3):
        graph.launch()
        gpu.run(u_e, work_e, dt_e, 2, 0.1)
        torch.cuda.synchronize()
        assert torch.equal(u_g, u_e), f"replay {rep} differs from dgamr_run"
    for _ in range(6):
        orc.step(u, 0.1)
    assert rel_diff(_host(u_g), u).max() <= TOL


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("bc", [W.PERIODIC, W.OUTFLOW])
def test_3d_thread_per_cell_conservative_mode_against_the_oracle(p, bc):
    """The thread-per-cell kernel's inline far side with mortar faces
    (conservative hanging mode, which the lane kernel does not take) on a
    three-level forest, against the oracle."""
    w = _forest(3, p, 4, 3, bc=bc)
    orc, gpu = make_pair(w, hanging=1)
    u = _physical_state(orc, w, seed=60 + p)
    got = _steps(gpu, u, 1, 3)
    for _ in range(3):
        orc.step(u, 0.1)
    assert rel_diff(got, u).max() <= TOL
