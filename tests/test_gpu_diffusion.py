"""GPU parity of the diffusion equation (Sec. 5.2, symmetric interior-penalty
DG with Dirichlet data from the exact exponential solution) against the
oracle: guard fill, residual at the forest's time, fused steps and runs
with the diffusive time step, the initial projection, and indicator-driven
regrids of the paper's diffusion case, in 2-D and 3-D with hanging faces.
FP64 bar 1e-12 relative (max |gpu - oracle| / max |oracle|)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import rel_diff

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
CFL = {1: 0.02, 2: 0.006, 3: 0.0025}


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _pair(dim, p, N, levels, bc=2, nu=0.7, avec=(-1.0, 1.0, 0.5)):
    G = _G()
    roots = (2, 2) if dim == 2 else (2, 2, 1)
    hi = (1.0, 1.0) if dim == 2 else (1.0, 1.0, 0.5)
    args = (dim, p, N, roots, (0.0,) * dim, hi, (bc,) * dim, levels)
    orc = O.Forest(*args, equation=O.EQ_DIFFUSION, nu=nu, avec=avec[:dim])
    gpu = G.Forest(*args, equation=G.EQ_DIFFUSION, nu=nu, exact_a=avec[:dim])
    rules = []
    if levels >= 2:
        rules.append(lambda keys: np.array([1 if k[0] == 0 else 0 for k in keys], np.int8))
    if levels >= 3:
        rules.append(lambda keys: np.array([1 if (k[0] == 0 and k[2] == 1 and k[3] == 1) else 0 for k in keys],
                                           np.int8))
    for rule in rules:
        orc.adapt(rule(orc.keys()))
        gpu.adapt(rule(gpu.keys()), torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))
    assert np.array_equal(orc.keys(), gpu.keys())
    return orc, gpu


CASES = [(2, 1, 6, 3), (2, 2, 8, 2), (2, 3, 4, 3), (3, 1, 4, 3), (3, 2, 4, 2), (3, 3, 4, 2)]


@pytest.mark.parametrize("dim,p,N,levels", CASES)
@pytest.mark.parametrize("bc", [0, 2])
def test_fill_residual_and_steps(dim, p, N, levels, bc):
    print(f"diffusion parity dim={dim} p={p} N={N} levels={levels} bc={bc}", flush=True)
    orc, gpu = _pair(dim, p, N, levels, bc)
    rng = np.random.default_rng(dim * 10 + p)
    u = orc.project_ic(O.IC_EXP, [])
    ud = gpu.project_ic(_G().IC_EXP, [])
    assert rel_diff(_host(ud), u).max() <= TOL
    u[:, :, 1:, :] += 0.05 * rng.standard_normal(u[:, :, 1:, :].shape)
    ud = _cuda(u)
    orc.time = gpu.time = 0.125
    gd = gpu.new_guard()
    gpu.fill_guardcells(ud, gd)
    g_ref = orc.fill_guards(u)
    assert np.abs(_host(gd) - g_ref).max() <= 1e-13 * max(1.0, np.abs(g_ref).max())
    rd = gpu.new_residual()
    gpu.dg_residual(ud, gd, rd)
    assert rel_diff(_host(rd), orc.residual(u, g_ref)).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, CFL[p])
        gpu.step(ud, work, dt, CFL[p])
        assert _host(dt)[0] == pytest.approx(dref, rel=1e-15)
    assert gpu.time == pytest.approx(orc.time, rel=1e-15)
    assert rel_diff(_host(ud), u).max() <= TOL
    for _ in range(4):
        orc.step(u, CFL[p])
    gpu.run(ud, work, dt, 4, CFL[p])
    assert rel_diff(_host(ud), u).max() <= TOL


def test_paper_diffusion_case_with_regrids():
    """Sec. 5.2's case over a short time window: one root on the unit
    square, 6x6-cell blocks, exp(-x + y + 2t) with Dirichlet data, levels
    2..4 refined by the block's largest cell average (above 3.0 refine,
    below 1.0 coarsen), regrid every 10 steps, started at t = 0.1 where the
    corner (0, 1) has grown above 3; GPU against the oracle leaf by leaf,
    and the leaf count changes."""
    G = _G()
    w = W.diffusion_2d()
    args = (w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level)
    orc = O.Forest(*args, equation=O.EQ_DIFFUSION, nu=w.nu, avec=w.exact_a)
    gpu = G.Forest(*args, equation=G.EQ_DIFFUSION, nu=w.nu, exact_a=w.exact_a)
    for rule in w.initial_refinement:
        orc.adapt(rule(w, orc.keys()))
        gpu.adapt(rule(w, gpu.keys()), torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))
    t0 = 0.1
    u = orc.project_ic(O.IC_EXP, [], t0)
    ud = gpu.project_ic(G.IC_EXP, [], t0)
    orc.time = gpu.time = t0
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    leaves = {orc.n_leaves}
    for step in range(40):
        if step % w.regrid_every == 0:
            eta = orc.indicator(u)
            np.testing.assert_allclose(_host(gpu.indicator(ud, work)), eta, rtol=1e-13)
            flags = W.regrid_flags(w, orc.keys(), eta)
            u = orc.adapt(flags, u)
            ud = gpu.adapt(flags, ud)
            work = gpu.new_work()
            assert np.array_equal(orc.keys(), gpu.keys())
            leaves.add(orc.n_leaves)
        orc.step(u, w.cfl)
        gpu.step(ud, work, dt, w.cfl)
    assert len(leaves) > 1
    assert rel_diff(_host(ud), u).max() <= TOL
    l1, l2 = orc.errors(u, O.IC_EXP, [], orc.time)
    assert l2[0] < 1e-3


def test_gpu_exact_solution_order():
    """The GPU path alone against the exact solution: observed L2 order
    p + 1 at p = 2 (oracle error norm of the GPU states)."""
    G = _G()
    errs = []
    for N in (4, 8):
        args = (2, 2, N, (1, 1), (0.0, 0.0), (1.0, 1.0), (2, 2), 1)
        gpu = G.Forest(*args, equation=G.EQ_DIFFUSION, nu=1.0, exact_a=(-1.0, 1.0))
        orc = O.Forest(*args, equation=O.EQ_DIFFUSION, nu=1.0, avec=(-1.0, 1.0))
        ud = gpu.project_ic(G.IC_EXP, [])
        work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
        T = 0.01
        n = int(math.ceil(T / (0.003 / N ** 2)))
        gpu.run(ud, work, dt, n, cfl=(T / n) * 2 * N ** 2)
        assert gpu.time == pytest.approx(T, rel=1e-12)
        errs.append(orc.errors(_host(ud), O.IC_EXP, [], T)[1][0])
    assert math.log2(errs[0] / errs[1]) >= 2.8, errs
