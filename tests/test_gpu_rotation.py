"""GPU parity on forests whose roots carry rotated local frames (Sec. 3.1
relative rotations, Sec. 3.5 guard fill K_d = R^n K_s / R^n S^i K_s /
R^n C(...)): the guard fill across rotated root faces (same level, coarser
and finer neighbours), the residual, fused and captured runs, the FP32
residual, the positivity limiter and the diffusion equation, against the
oracle's rotated frames, element by element.  FP64 bar 1e-12 relative."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import rel_diff, rel_diff_floored

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _pair(dim, p, N, frames, levels=3, precision=0, limiter=False, equation=0, bc=0):
    G = _G()
    roots = (2, 2) if dim == 2 else (2, 2, 2)
    L = 10.0 if dim == 2 else 4.0
    args = (dim, p, N, roots, (0.0,) * dim, (L,) * dim, (bc,) * dim, levels)
    kw_o, kw_g = {}, {}
    if equation == 2:
        kw_o = dict(equation=O.EQ_DIFFUSION, nu=0.8, avec=(-1.0, 0.5, 0.25)[:dim])
        kw_g = dict(equation=G.EQ_DIFFUSION, nu=0.8, exact_a=(-1.0, 0.5, 0.25)[:dim])
    elif equation == 1:
        kw_o = dict(equation=O.EQ_ADVECTION, velocity=(1.0, 0.5, 0.25))
        kw_g = dict(equation=G.EQ_ADVECTION, velocity=(1.0, 0.5, 0.25))
    orc = O.Forest(*args, **kw_o)
    gpu = G.Forest(*args, precision=precision, limiter=G.LIMITER_POSITIVITY if limiter else G.LIMITER_NONE, **kw_g)
    orc.set_frames(frames)
    gpu.set_root_frames(frames)
    # root 0 refined, then its child touching root 1 refined again: hanging
    # faces (coarse-fine and fine-coarse) across rotated root faces
    flags = np.zeros(orc.n_leaves, np.int8)
    flags[0] = 1
    orc.adapt(flags)
    gpu.adapt(flags, torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))
    if levels >= 3:
        flags = np.zeros(orc.n_leaves, np.int8)
        flags[1] = 1
        orc.adapt(flags)
        gpu.adapt(flags, torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))
    assert np.array_equal(orc.keys(), gpu.keys())
    return orc, gpu


def _frames(dim, seed):
    rng = np.random.default_rng(seed)
    n = 4 if dim == 2 else 8
    return [int(x) for x in rng.integers(0, 4 if dim == 2 else 24, n)]


CASES = [(2, 1, 4), (2, 2, 6), (2, 3, 4), (3, 1, 2), (3, 2, 4), (3, 3, 2)]


@pytest.mark.parametrize("dim,p,N", CASES)
@pytest.mark.parametrize("seed", [1, 2])
def test_rotated_fill_residual_and_steps(dim, p, N, seed):
    frames = _frames(dim, seed)
    print(f"rotated parity dim={dim} p={p} N={N} frames={frames}", flush=True)
    orc, gpu = _pair(dim, p, N, frames)
    prm = [3.0, 4.0, 6.0, 0.7, -0.4, 10.0, 10.0] if dim == 2 else [2.0, 1.5, 2.5, 0.5, 0.3, 4.0, 4.0]
    u = orc.project_ic(O.IC_VORTEX, prm)
    ud = gpu.project_ic(_G().IC_VORTEX, prm)
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
    assert rel_diff_floored(_host(rd), orc.residual(u, g_ref), 1e-3).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12, atol=1e-12)
    # run (dt per step) and a captured run equal the same steps
    ua, ub = ud.clone(), ud.clone()
    for _ in range(2):
        orc.step(u, 0.1)
    gpu.run(ua, work, dt, 2, 0.1)
    assert rel_diff_floored(_host(ua), u, 1e-3).max() <= TOL
    g = gpu.capture_run(ub, gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda"), 2, 0.1)
    g.launch()
    assert rel_diff(_host(ub), _host(ua)).max() <= 1e-14


def test_rotated_fp32_residual():
    frames = _frames(3, 5)
    G = _G()
    orc, gpu = _pair(3, 2, 4, frames, precision=G.FP32)
    prm = [2.0, 1.5, 2.5, 0.5, 0.3, 4.0, 4.0]
    u = orc.project_ic(O.IC_VORTEX, prm)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= 1e-5


@pytest.mark.parametrize("p,N", [(1, 4), (2, 6), (3, 4)])
@pytest.mark.parametrize("variant", [0, 1])
def test_rotated_2d_steps_in_both_stage_kernels(p, N, variant):
    """The fused stage reading the far side from the rotated guard fill, in
    both 2-D stage kernels (one lane per cell and variable; one thread per
    cell), on a three-level forest."""
    G = _G()
    frames = _frames(2, 3)
    orc, gpu = _pair(2, p, N, frames)
    gpu.set_tuning(G.TUNE_STAGE_VARIANT, variant)
    prm = [3.0, 4.0, 6.0, 0.7, -0.4, 10.0, 10.0]
    u = orc.project_ic(O.IC_VORTEX, prm)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(4):
        dref = orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL


@pytest.mark.parametrize("dim", [2, 3])
def test_rotated_blast_with_limiter(dim):
    """A pressure jump with the positivity limiter on rotated roots."""
    frames = _frames(dim, 7)
    orc, gpu = _pair(dim, 2, 4, frames, limiter=True, levels=2)
    u = orc.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1e-3])
    u[0, dim + 1, 0, :] = 1e3 / 0.4  # one leaf at high pressure, the rest near vacuum
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        orc.step(u, 0.1, limiter=True)
        gpu.step(ud, work, dt, 0.1)
    assert rel_diff_floored(_host(ud), u, 1e-3).max() <= TOL
    assert gpu.check_state(ud, work) == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_rotated_diffusion(dim):
    frames = _frames(dim, 11)
    G = _G()
    orc, gpu = _pair(dim, 2, 4, frames, equation=2, bc=2, levels=2)
    u = orc.project_ic(O.IC_EXP, [])
    ud = gpu.project_ic(G.IC_EXP, [])
    assert rel_diff(_host(ud), u).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        orc.step(u, 0.006)
        gpu.step(ud, work, dt, 0.006)
    assert rel_diff(_host(ud), u).max() <= TOL


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_rotated_scalar_convection(dim, p):
    """Scalar convection on rotated roots (the velocity along each root's
    local axes), hanging faces across rotated root faces: projection,
    fused steps with the fill of the rotated guard cells, dt, totals."""
    G = _G()
    frames = _frames(dim, 13 + p)
    orc, gpu = _pair(dim, p, 4 if dim == 2 else 2, frames, equation=1)
    L = 10.0 if dim == 2 else 4.0
    prm = [1.0, L, L, L]
    u = orc.project_ic(O.IC_COSINE, prm)
    ud = gpu.project_ic(G.IC_COSINE, prm)
    assert rel_diff(_host(ud), u).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(4):
        dref = orc.step(u, 0.2)
        gpu.step(ud, work, dt, 0.2)
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff(_host(ud), u).max() <= TOL
    np.testing.assert_allclose(_host(gpu.conserved_totals(ud, work)), orc.totals(u), rtol=1e-12, atol=1e-12)


def test_frames_refused_where_not_defined():
    G = _G()
    f = G.Forest(2, 1, 4, (2, 1), (0.0, 0.0), (2.0, 2.0), (0, 0), 2)
    with pytest.raises(G.DgamrError):
        f.set_root_frames([1, 0])  # root edges 1 x 2
    g = G.Forest(2, 1, 4, (2, 2), (0.0, 0.0), (2.0, 2.0), (0, 0), 2, hanging=G.HANG_CONSERVATIVE)
    with pytest.raises(G.DgamrError):
        g.set_root_frames([1, 0, 0, 0])
    h = G.Forest(2, 1, 4, (2, 2), (0.0, 0.0), (2.0, 2.0), (0, 0), 2)
    h.adapt(np.array([1, 0, 0, 0], np.int8), torch.zeros(h.state_shape(), dtype=torch.float64, device="cuda"))
    with pytest.raises(G.DgamrError):
        h.set_root_frames([1, 0, 0, 0])  # after a refinement
