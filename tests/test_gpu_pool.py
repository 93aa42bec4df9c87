"""GPU tests of pools (many forests stepped together by the same stage
kernels): every member's result equals the same forest stepped alone
(bitwise: a member's arithmetic does not depend on the other members; a
different slab height changes it only at rounding level), members admitted and released between steps
(continuous batching), HIP-graph replay against eager steps, the
autotuner, and agreement with the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import make_pair, rel_diff, rel_diff_floored

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _vortex(name, dim, p, N, roots, edge, eps, centre, levels=1, refine_tree0=False):
    hi = tuple(edge * r for r in roots)
    prm = [eps, centre[0], centre[1], 1.0, 1.0, hi[0], hi[1]]
    w = W.Workload(name, dim, p, N, roots, (0.0,) * dim, hi, (W.PERIODIC,) * dim, levels, W.IC_VORTEX, prm, 1)
    if refine_tree0:
        w.initial_refinement = [lambda w_, keys: np.array([1 if k[0] == 0 else 0 for k in keys], np.int8)]
    return w


def _gpu_forest(w, precision=None, hanging=0, limiter=False):
    G = _G()
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                 precision=G.FP64 if precision is None else precision, hanging=hanging,
                 limiter=G.LIMITER_POSITIVITY if limiter else G.LIMITER_NONE)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    return f


def _solo(w, cfl, steps, precision=None, hanging=0, limiter=False):
    """The forest stepped alone through dgamr_step with the thread-per-cell
    stage kernel (the pool's kernel)."""
    G = _G()
    f = _gpu_forest(w, precision, hanging, limiter)
    f.set_tuning(G.TUNE_STAGE_VARIANT, 1)
    u = f.project_ic(G.IC_VORTEX, w.ic_params)
    work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        f.step(u, work, dt, cfl)
    return _host(u)


def _members_2d(p):
    return [(_vortex("a", 2, p, 8, (2, 2), 2.0, 3.0, (2.0, 2.0), levels=2, refine_tree0=True), 0.1),
            (_vortex("b", 2, p, 8, (1, 1), 10.0, 5.0, (5.0, 5.0)), 0.05),
            (_vortex("c", 2, p, 8, (3, 2), 2.5, 2.0, (3.0, 2.0)), 0.2)]


def _admit_all(pool, members, precision=None, hanging=0, limiter=False):
    G = _G()
    out = []
    for w, cfl in members:
        f = _gpu_forest(w, precision, hanging, limiter)
        mid, first = pool.admit(f, cfl)
        f.project_ic(G.IC_VORTEX, w.ic_params, u=pool.view(first, f.n_leaves))
        out.append((f, mid, first))
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_pool_members_equal_solo_runs(p):
    G = _G()
    members = _members_2d(p)
    pool = G.Pool(2, p, 8, capacity_leaves=64, max_members=8)
    adm = _admit_all(pool, members)
    steps = 4
    for _ in range(steps):
        pool.step()
    for (w, cfl), (f, mid, first) in zip(members, adm):
        got = _host(pool.view(first, f.n_leaves))
        assert np.array_equal(got, _solo(w, cfl, steps)), f"member {w.name} differs from its solo run"
    # and the AMR member against the oracle
    w, cfl = members[0]
    orc, _ = make_pair(w)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    for _ in range(steps):
        orc.step(u, cfl)
    f, _, first = adm[0]
    assert rel_diff(_host(pool.view(first, f.n_leaves)), u).max() <= 1e-12


def test_pool_continuous_batching():
    """Members join and leave between steps; each result equals its solo
    run, and a released range is reused."""
    G = _G()
    wa, wb, wc = (m[0] for m in _members_2d(2))
    pool = G.Pool(2, 2, 8, capacity_leaves=12, max_members=2)
    fa = _gpu_forest(wa)
    ma, sa = pool.admit(fa, 0.1)
    fa.project_ic(G.IC_VORTEX, wa.ic_params, u=pool.view(sa, fa.n_leaves))
    for _ in range(3):
        pool.step()
    fb = _gpu_forest(wb)
    mb, sb = pool.admit(fb, 0.05)
    fb.project_ic(G.IC_VORTEX, wb.ic_params, u=pool.view(sb, fb.n_leaves))
    fc = _gpu_forest(wc)
    with pytest.raises(G.DgamrError) as e:  # 6 leaves do not fit beside 7 + 1
        pool.admit(fc, 0.2)
    assert e.value.code == G.EFULL
    for _ in range(3):
        pool.step()
    a_out = _host(pool.view(sa, fa.n_leaves)).copy()
    pool.release(ma)
    mc, sc = pool.admit(fc, 0.2)
    assert sc == sa  # first fit reuses the released range
    fc.project_ic(G.IC_VORTEX, wc.ic_params, u=pool.view(sc, fc.n_leaves))
    for _ in range(2):
        pool.step()
    assert pool.stats() == (fb.n_leaves + fc.n_leaves, 2)
    assert np.array_equal(a_out, _solo(wa, 0.1, 6))
    assert np.array_equal(_host(pool.view(sb, fb.n_leaves)), _solo(wb, 0.05, 5))
    assert np.array_equal(_host(pool.view(sc, fc.n_leaves)), _solo(wc, 0.2, 2))


def test_graph_replay_matches_eager_steps():
    G = _G()
    pools, eager = [], []
    for p in (1, 3):
        for lst in (pools, eager):
            pool = G.Pool(2, p, 8, capacity_leaves=64, max_members=4)
            _admit_all(pool, _members_2d(p))
            lst.append(pool)
    torch.cuda.synchronize()
    g = G.Graph(pools, nsteps=2)
    scratch = torch.rand(1 << 20, device="cuda")
    for rep in range(3):
        g.launch()
        for pool in eager:
            for _ in range(2):
                pool.step()
        scratch.mul_(1.0001)  # eager work between replays
        torch.cuda.synchronize()
        for a, b in zip(pools, eager):
            assert torch.equal(a.u, b.u), f"replay {rep} differs from eager steps"
    # a changed pool invalidates the graph
    extra = _gpu_forest(_members_2d(1)[1][0])
    pools[0].admit(extra, 0.1)
    with pytest.raises(G.DgamrError) as e:
        g.launch()
    assert e.value.code == G.ESTATE


def test_autotune_keeps_results():
    G = _G()
    members = _members_2d(2)
    ref = G.Pool(2, 2, 8, capacity_leaves=64, max_members=8)
    _admit_all(ref, members)
    tuned = G.Pool(2, 2, 8, capacity_leaves=64, max_members=8)
    _admit_all(tuned, members)
    variant, rows, grid, us = tuned.autotune()
    assert variant in (0, 1) and rows in (8, 4, 2, 1) and grid >= 0 and us > 0
    # a persistent grid walks the same items: bitwise the same result
    tuned.set_shape(8, 4)
    tuned.step()
    ref.step()
    assert torch.equal(tuned.u, ref.u), "a persistent grid changes the result"
    # another slab height computes slab-edge faces from memory instead of
    # LDS: the same arithmetic up to rounding
    for shape in [(rows, grid), (2, 0), (1, 256)]:
        tuned.set_shape(*shape)
        tuned.step()
        ref.step()
        assert rel_diff(_host(tuned.u), _host(ref.u)).max() <= 1e-14, f"shape {shape}"
    # the autotuner's own choice (which may be the lane-per-variable kernel)
    tuned.autotune()
    tuned.step()
    ref.step()
    assert rel_diff(_host(tuned.u), _host(ref.u)).max() <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_pool_persistent_grid(dim):
    """FP32 pools (degree 2: the volume integral on the matrix cores, whose
    per-wave LDS regions alias the face exchange of the previous work item)
    on a persistent grid of fewer workgroups than items: bitwise equal to one
    workgroup per item."""
    G = _G()
    if dim == 2:
        members = _members_2d(2)
        args, shape = (2, 2, 8), (8, 3)
    else:
        members = [(_vortex("a3", 3, 2, 4, (2, 2, 1), 2.0, 3.0, (2.0, 2.0), levels=2, refine_tree0=True), 0.1),
                   (_vortex("b3", 3, 2, 4, (1, 2, 2), 2.5, 2.0, (1.0, 2.0)), 0.15)]
        args, shape = (3, 2, 4), (4, 3)
    pools = []
    for grid in (0, shape[1]):
        pool = G.Pool(*args, capacity_leaves=64, max_members=8, precision=G.FP32)
        _admit_all(pool, members, precision=G.FP32)
        pool.set_shape(shape[0], grid)
        for _ in range(3):
            pool.step()
        pools.append(pool)
    assert torch.equal(pools[0].u, pools[1].u), "a persistent grid changes the FP32 result"


@pytest.mark.parametrize("precision,limiter", [(0, False), (1, False), (0, True)])
def test_pool_3d_members(precision, limiter):
    G = _G()
    members = [(_vortex("a3", 3, 2, 4, (2, 2, 1), 2.0, 3.0, (2.0, 2.0), levels=2, refine_tree0=True), 0.1),
               (_vortex("b3", 3, 2, 4, (1, 2, 2), 2.5, 2.0, (1.0, 2.0)), 0.15)]
    pool = G.Pool(3, 2, 4, capacity_leaves=64, max_members=4, precision=precision,
                  limiter=G.LIMITER_POSITIVITY if limiter else G.LIMITER_NONE)
    adm = _admit_all(pool, members, precision=precision, limiter=limiter)
    for _ in range(3):
        pool.step()
    for (w, cfl), (f, mid, first) in zip(members, adm):
        got = _host(pool.view(first, f.n_leaves))
        assert np.array_equal(got, _solo(w, cfl, 3, precision=precision, limiter=limiter))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_pool_3d_lane_kernel(p):
    """3-D members stepped by the lane-per-(cell, variable) kernel over the
    pool's work list with per-member dt agree with their solo runs (thread
    per cell) to rounding; the autotuner's choice agrees too."""
    G = _G()
    members = [(_vortex("a3", 3, p, 4, (2, 2, 1), 2.0, 3.0, (2.0, 2.0), levels=2, refine_tree0=True), 0.1),
               (_vortex("b3", 3, p, 4, (1, 2, 2), 2.5, 2.0, (1.0, 2.0)), 0.15)]
    for rows in (2, 4, 0):
        pool = G.Pool(3, p, 4, capacity_leaves=64, max_members=4)
        adm = _admit_all(pool, members)
        pool.set_lanes(rows)
        for _ in range(3):
            pool.step()
        for (w, cfl), (f, mid, first) in zip(members, adm):
            got = _host(pool.view(first, f.n_leaves))
            assert rel_diff_floored(got, _solo(w, cfl, 3), floor=1e-2).max() <= 1e-13, f"rows {rows}, member {w.name}"
    with pytest.raises(G.DgamrError):
        pool.set_lanes(1)  # a one-layer slab of a 4-layer block
    ref = G.Pool(3, p, 4, capacity_leaves=64, max_members=4)
    _admit_all(ref, members)
    tuned = G.Pool(3, p, 4, capacity_leaves=64, max_members=4)
    _admit_all(tuned, members)
    variant, rows, grid, us = tuned.autotune()
    assert variant in (0, 1) and us > 0
    for _ in range(2):
        tuned.step()
        ref.step()
    assert rel_diff_floored(_host(tuned.u), _host(ref.u), floor=1e-2).max() <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_run_capture_replays_equal_run(dim):
    """A single forest's captured run (CFL step inside the graph) replayed
    several times, with eager work between replays, equals dgamr_run."""
    G = _G()
    if dim == 2:
        w = _vortex("g2", 2, 2, 8, (2, 2), 2.0, 3.0, (2.0, 2.0), levels=2, refine_tree0=True)
    else:
        w = _vortex("g3", 3, 1, 4, (2, 2, 1), 2.0, 3.0, (2.0, 2.0), levels=2, refine_tree0=True)
    f = _gpu_forest(w)
    u_g = f.project_ic(G.IC_VORTEX, w.ic_params)
    u_e = u_g.clone()
    work_g, work_e = f.new_work(), f.new_work()
    dt_g, dt_e = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2))
    graph = f.capture_run(u_g, work_g, dt_g, 3, 0.1)
    scratch = torch.rand(1 << 18, device="cuda")
    for rep in range(3):
        graph.launch()
        f.run(u_e, work_e, dt_e, 3, 0.1)
        scratch.add_(1.0)
        torch.cuda.synchronize()
        assert torch.equal(u_g, u_e), f"replay {rep} differs from dgamr_run"
        assert torch.equal(dt_g, dt_e)
    f.adapt(np.zeros(f.n_leaves, np.int8), u_g)  # a (trivial) refinement invalidates the graph
    with pytest.raises(G.DgamrError) as e:
        graph.launch()
    assert e.value.code == G.ESTATE
