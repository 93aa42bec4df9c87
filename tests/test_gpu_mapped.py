"""GPU parity on bilinear and trilinear root blocks (Sec. 3.3, Eq. 6): distorted
root grids, periodic and outflow, with hanging faces, against the oracle's
bilinear blocks element by element: the initial projection (full mass
matrix), the guard fill (reference-space copy, split, combine), the
residual with the metric terms, fused steps with the CFL rate of the
physical cells, runs and captured runs, totals over the physical cells, a
regrid, scalar convection, and the positivity limiter about the physical
cell mean (alone and fused with the stages).  FP64 bar 1e-12 relative per variable for
states; 4e-12 for the residual of a perturbed state, which is M^-1 of the
volume and face sums: the solve with a cell's full mass matrix multiplies
the sums' rounding by up to its condition number (25 for the Legendre mass
of the reference cell at p = 2, 100 at p = 3, more on distorted cells),
against the diagonal mass of box cells."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import rel_diff, rel_diff_floored
from tests.test_oracle_mapped import PRM3, box_nodes3, distorted_nodes, distorted_nodes3

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_RES = 4e-12
PRM = [3.0, 5.0, 5.0, 0.7, -0.4, 10.0, 10.0]


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _adapt_both(orc, gpu, which):
    flags = np.zeros(orc.n_leaves, np.int8)
    flags[which] = 1
    orc.adapt(flags)
    gpu.adapt(flags, torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))


def _pair(p, N, bc, seed, equation=0, levels=3):
    G = _G()
    roots, lo, hi = (3, 3), (0.0, 0.0), (10.0, 10.0)
    args = (2, p, N, roots, lo, hi, (bc, bc), max(levels, 2))
    if equation == 1:
        orc = O.Forest(*args, equation=O.EQ_ADVECTION, velocity=(1.0, 0.5, 0.0))
        gpu = G.Forest(*args, equation=G.EQ_ADVECTION, velocity=(1.0, 0.5, 0.0))
    else:
        orc, gpu = O.Forest(*args), G.Forest(*args)
    nodes = distorted_nodes(roots, lo, hi, 0.2, seed=seed)
    orc.set_nodes(nodes)
    gpu.set_root_nodes(nodes)
    # the centre root refined, then one of its children: hanging faces of
    # both kinds between distorted roots
    if levels >= 2:
        _adapt_both(orc, gpu, 4)
    if levels >= 3:
        _adapt_both(orc, gpu, 5)
    assert np.array_equal(orc.keys(), gpu.keys())
    return orc, gpu


CASES = [(1, 4), (2, 4), (2, 6), (3, 4), (0, 4)]


@pytest.mark.parametrize("p,N", CASES)
@pytest.mark.parametrize("bc", [0, 1])
def test_mapped_fill_residual_and_steps(p, N, bc):
    print(f"bilinear parity p={p} N={N} bc={bc}", flush=True)
    orc, gpu = _pair(p, N, bc, seed=p + 10 * N)
    G = _G()
    u = orc.project_ic(O.IC_VORTEX, PRM)
    ud = gpu.project_ic(G.IC_VORTEX, PRM)
    assert rel_diff(_host(ud), u).max() <= TOL
    rng = np.random.default_rng(p + N)
    if p > 0:
        u[:, :, 1:, :] += 0.01 * rng.standard_normal(u[:, :, 1:, :].shape)
    ud = _cuda(u)
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    g_ref = orc.fill_guards(u)
    assert np.abs(_host(gd) - g_ref).max() <= 1e-13 * np.abs(g_ref).max()
    rd = gpu.new_residual()
    gpu.dg_residual(ud, gd, rd)
    assert rel_diff(_host(rd), orc.residual(u, g_ref)).max() <= TOL_RES
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff(_host(ud), u).max() <= TOL
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12, atol=1e-12)
    ua, ub = ud.clone(), ud.clone()
    for _ in range(2):
        orc.step(u, 0.1)
    gpu.run(ua, work, dt, 2, 0.1)
    assert rel_diff(_host(ua), u).max() <= TOL
    g = gpu.capture_run(ub, gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda"), 2, 0.1)
    for _ in range(1):
        g.launch()
    assert rel_diff(_host(ub), _host(ua)).max() <= 1e-14


def test_mapped_conservation_and_regrid():
    """Periodic distorted roots: on the conforming forest the GPU totals are
    conserved over steps (every variable); then a regrid (refine one leaf,
    coarsen a family; reference-space inheritance) and more steps with
    hanging faces, against the oracle."""
    G = _G()
    orc0, gpu0 = _pair(2, 4, 0, seed=3, levels=1)
    ud0 = gpu0.project_ic(G.IC_VORTEX, PRM)
    work0, dt = gpu0.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = _host(gpu0.conserved_totals(ud0, work0))
    for _ in range(3):
        gpu0.step(ud0, work0, dt, 0.1)
    np.testing.assert_allclose(_host(gpu0.conserved_totals(ud0, work0)), t0, rtol=1e-13, atol=1e-12)
    orc, gpu = _pair(2, 4, 0, seed=3)
    u = orc.project_ic(O.IC_VORTEX, PRM)
    ud = gpu.project_ic(G.IC_VORTEX, PRM)
    work = gpu.new_work()
    for _ in range(3):
        orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
    assert rel_diff(_host(ud), u).max() <= TOL
    n0 = orc.n_leaves
    flags = np.zeros(n0, np.int8)
    flags[0] = 1
    keys = orc.keys()
    fine = [i for i, k in enumerate(keys) if k[1] == 3]
    flags[fine] = -1  # the level-3 family coarsens again
    u = orc.adapt(flags, u)
    ud = gpu.adapt(flags, ud)
    assert np.array_equal(orc.keys(), gpu.keys())
    assert orc.keys().shape != keys.shape or not np.array_equal(orc.keys(), keys), "the regrid changed nothing"
    assert rel_diff(_host(ud), u).max() <= TOL
    work = gpu.new_work()
    for _ in range(3):
        orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
    assert rel_diff(_host(ud), u).max() <= TOL


@pytest.mark.parametrize("p", [1, 2])
def test_mapped_scalar_convection(p):
    orc, gpu = _pair(p, 4, 0, seed=9, equation=1)
    G = _G()
    prm = [1.0, 10.0, 10.0, 10.0]
    u = orc.project_ic(O.IC_COSINE, prm)
    ud = gpu.project_ic(G.IC_COSINE, prm)
    assert rel_diff(_host(ud), u).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(4):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff(_host(ud), u).max() <= TOL
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12, atol=1e-12)


def test_mapped_refusals():
    G = _G()
    roots, lo, hi = (2, 2), (0.0, 0.0), (1.0, 1.0)
    nodes = distorted_nodes(roots, lo, hi, 0.1, seed=1)
    for kw in (dict(precision=G.FP32), dict(hanging=G.HANG_CONSERVATIVE)):
        f = G.Forest(2, 1, 4, roots, lo, hi, (0, 0), 2, **kw)
        with pytest.raises(G.DgamrError) as e:
            f.set_root_nodes(nodes)
        assert e.value.code == G.EUNSUPPORTED
    f = G.Forest(2, 1, 4, roots, lo, hi, (0, 0), 2)
    bad = nodes.copy()
    bad[1, 1] = [1.2, 1.2]  # folds the roots around the centre node
    with pytest.raises(G.DgamrError) as e:
        f.set_root_nodes(bad)
    assert e.value.code == G.EINVAL
    f.set_root_nodes(nodes)
    g = G.Forest(3, 3, 2, (1, 1, 1), (0.0,) * 3, (1.0,) * 3, (0, 0, 0), 1)
    with pytest.raises(G.DgamrError) as e:
        g.set_root_nodes(box_nodes3((1, 1, 1), (0.0,) * 3, (1.0,) * 3))
    assert e.value.code == G.EUNSUPPORTED  # trilinear blocks at degree <= 2


CASES3 = [(1, 2), (2, 2), (1, 4)]


@pytest.mark.parametrize("p,N", CASES3)
@pytest.mark.parametrize("bc", [0, 1])
def test_trilinear_fill_residual_and_steps(p, N, bc):
    """2x2x2 distorted roots, root 0 refined and then one of its children:
    the same checks as in 2-D, against the oracle's trilinear blocks."""
    print(f"trilinear parity p={p} N={N} bc={bc}", flush=True)
    G = _G()
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (4.0,) * 3
    args = (3, p, N, roots, lo, hi, (bc,) * 3, 3)
    orc, gpu = O.Forest(*args), G.Forest(*args)
    nodes = distorted_nodes3(roots, lo, hi, 0.15, seed=p + 10 * N + bc)
    orc.set_nodes(nodes)
    gpu.set_root_nodes(nodes)
    _adapt_both(orc, gpu, 0)
    _adapt_both(orc, gpu, 1)
    assert np.array_equal(orc.keys(), gpu.keys())
    u = orc.project_ic(O.IC_VORTEX, PRM3)
    ud = gpu.project_ic(G.IC_VORTEX, PRM3)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    rng = np.random.default_rng(p + N + bc)
    u[:, :, 1:, :] += 0.01 * rng.standard_normal(u[:, :, 1:, :].shape)
    ud = _cuda(u)
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    g_ref = orc.fill_guards(u)
    assert np.abs(_host(gd) - g_ref).max() <= 1e-13 * np.abs(g_ref).max()
    rd = gpu.new_residual()
    gpu.dg_residual(ud, gd, rd)
    assert rel_diff_floored(_host(rd), orc.residual(u, g_ref), 1e-3).max() <= TOL_RES
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12, atol=1e-12)


def test_trilinear_scalar_convection():
    G = _G()
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (1.0,) * 3
    args = (3, 1, 2, roots, lo, hi, (0, 0, 0), 2)
    orc = O.Forest(*args, equation=O.EQ_ADVECTION, velocity=(1.0, 0.5, 0.25))
    gpu = G.Forest(*args, equation=G.EQ_ADVECTION, velocity=(1.0, 0.5, 0.25))
    nodes = distorted_nodes3(roots, lo, hi, 0.15, seed=4)
    orc.set_nodes(nodes)
    gpu.set_root_nodes(nodes)
    _adapt_both(orc, gpu, 3)
    prm = [1.0, 1.0, 1.0, 1.0]
    u = orc.project_ic(O.IC_COSINE, prm)
    ud = gpu.project_ic(G.IC_COSINE, prm)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff(_host(ud), u).max() <= TOL


# ---------------------------------------------------------------- rotated frames on bilinear / trilinear roots

def _frames(dim, n, seed):
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(0, 4 if dim == 2 else 24, n)]


def _rotated_mapped_checks(orc, gpu, prm, steps, seed):
    G = _G()
    u = orc.project_ic(O.IC_VORTEX, prm)
    ud = gpu.project_ic(G.IC_VORTEX, prm)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    rng = np.random.default_rng(seed)
    u[:, :, 1:, :] += 0.01 * rng.standard_normal(u[:, :, 1:, :].shape)
    ud = _cuda(u)
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    g_ref = orc.fill_guards(u)
    assert np.abs(_host(gd) - g_ref).max() <= 1e-13 * np.abs(g_ref).max()
    rd = gpu.new_residual()
    gpu.dg_residual(ud, gd, rd)
    assert rel_diff_floored(_host(rd), orc.residual(u, g_ref), 1e-3).max() <= TOL_RES
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("p,N", [(1, 4), (2, 4), (3, 4)])
@pytest.mark.parametrize("bc", [0, 1])
def test_rotated_frames_on_bilinear_roots(p, N, bc):
    """Distorted 3x3 roots with seeded frames (set after the nodes), the
    centre root and one of its children refined: initial projection, fill
    (the modes turned, the momentum kept along the global axes), residual,
    steps and totals against the oracle."""
    print(f"rotated bilinear parity p={p} N={N} bc={bc}", flush=True)
    G = _G()
    roots, lo, hi = (3, 3), (0.0, 0.0), (10.0, 10.0)
    args = (2, p, N, roots, lo, hi, (bc, bc), 3)
    orc, gpu = O.Forest(*args), G.Forest(*args)
    nodes = distorted_nodes(roots, lo, hi, 0.2, seed=p + 3 * bc)
    frames = _frames(2, 9, seed=p + N + bc)
    orc.set_nodes(nodes)
    gpu.set_root_nodes(nodes)
    orc.set_frames(frames)
    gpu.set_root_frames(frames)
    _adapt_both(orc, gpu, 4)
    _adapt_both(orc, gpu, 5)
    assert np.array_equal(orc.keys(), gpu.keys())
    _rotated_mapped_checks(orc, gpu, PRM, 3, seed=p + bc)


@pytest.mark.parametrize("p,N", [(1, 2), (2, 2)])
def test_rotated_frames_on_trilinear_roots(p, N):
    """Distorted 2x2x2 roots with seeded frames (set before the nodes),
    root 0 refined: the same checks in 3-D."""
    print(f"rotated trilinear parity p={p} N={N}", flush=True)
    G = _G()
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (4.0,) * 3
    args = (3, p, N, roots, lo, hi, (0, 0, 0), 2)
    orc, gpu = O.Forest(*args), G.Forest(*args)
    frames = _frames(3, 8, seed=40 + p)
    orc.set_frames(frames)
    gpu.set_root_frames(frames)
    nodes = distorted_nodes3(roots, lo, hi, 0.15, seed=p + 7)
    orc.set_nodes(nodes)
    gpu.set_root_nodes(nodes)
    _adapt_both(orc, gpu, 0)
    assert np.array_equal(orc.keys(), gpu.keys())
    _rotated_mapped_checks(orc, gpu, PRM3, 2, seed=p)


def _blast(orc, dim, seed):
    """Near-vacuum pressure with a high-pressure leaf, random higher energy
    modes of 0.6 and density modes of 0.05 times the cell's mode 0: the
    pressure is negative at limiter points of most cells, and the density
    stays well above zero (a density limited down to eps at a point gives
    sound speeds there far above the CFL rate of the cell means, and the
    run blows up alike in both codes)."""
    u = orc.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1e-3])
    u[0, dim + 1, 0, :] = 1e3 / 0.4
    rng = np.random.default_rng(seed)
    amp = np.zeros(dim + 2)
    amp[0], amp[dim + 1] = 0.05, 0.6
    u[:, :, 1:, :] += amp[None, :, None, None] * rng.standard_normal(u[:, :, 1:, :].shape) * np.abs(u[:, :, :1, :])
    return u


@pytest.mark.parametrize("dim,p,N", [(2, 1, 4), (2, 2, 4), (2, 3, 4), (3, 1, 2), (3, 2, 2)])
def test_mapped_limiter_alone_and_fused(dim, p, N):
    """The positivity limiter on distorted roots with hanging faces, about
    each cell's mean over the physical cell: the limiter alone, and fused
    with the stages of limited steps."""
    print(f"mapped limiter dim={dim} p={p} N={N}", flush=True)
    G = _G()
    if dim == 2:
        roots, lo, hi = (3, 3), (0.0, 0.0), (10.0, 10.0)
        nodes = distorted_nodes(roots, lo, hi, 0.2, seed=p)
    else:
        roots, lo, hi = (2, 2, 2), (0.0,) * 3, (4.0,) * 3
        nodes = distorted_nodes3(roots, lo, hi, 0.15, seed=p)
    args = (dim, p, N, roots, lo, hi, (1,) * dim, 3)
    orc, gpu = O.Forest(*args), G.Forest(*args, limiter=G.LIMITER_POSITIVITY)
    orc.set_nodes(nodes)
    gpu.set_root_nodes(nodes)
    _adapt_both(orc, gpu, 0)
    _adapt_both(orc, gpu, 1)
    u = _blast(orc, dim, seed=p + N)
    ud = _cuda(u)
    u0 = u.copy()
    orc.limit(u)
    assert (np.abs(u - u0).max(axis=(1, 2)) > 0).mean() > 0.25  # the limiter acts on many cells
    gpu.limit_positivity(ud)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, 0.1, limiter=True)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    # the states of limited steps at the residual's bar: every stage's solve
    # with the cell's full mass matrix amplifies the rounding of its sums
    # (see TOL_RES), and the limiter's scale theta = (p(mean) - eps) /
    # (p(mean) - p(U)) carries it into every mode of the limited cells
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL_RES
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12,
                               atol=1e-12 * np.abs(orc.totals(u)).max())
    assert gpu.check_state(ud, work) == 0
    # run (dt per step) and a captured run equal the same limited steps
    ua, ub = ud.clone(), ud.clone()
    for _ in range(2):
        orc.step(u, 0.1, limiter=True)
    gpu.run(ua, work, dt, 2, 0.1)
    assert rel_diff_floored(_host(ua), u, 1e-3).max() <= TOL_RES
    g = gpu.capture_run(ub, gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda"), 2, 0.1)
    g.launch()
    assert rel_diff(_host(ub), _host(ua)).max() <= 1e-14
