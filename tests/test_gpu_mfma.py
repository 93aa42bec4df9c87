"""The FP32 residual with its volume integral on the matrix cores
(v_mfma_f32_16x16x4f32, FP32 accumulation; degree >= 2, stage workgroups
of whole waves) against the FP64 oracle and against the same FP32 kernel
with the volume integral on the vector unit (tuning knob DGAMR_TUNE_MFMA,
off by default).
Tolerances as in test_gpu_fp32: 1e-4 relative per variable for a residual
(a signed sum of at most d N_q + 2d N_f rounded products), 1e-5 for states
after a few stages.  The two FP32 variants sum in different orders, so
their results differ in the last bits: that they differ at all shows the
matrix-core path ran."""
import numpy as np
import pytest

import oracle as O
from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import make_pair, rel_diff

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_RES32 = 1e-4
TOL_STATE32 = 1e-5  # the bar of the FP32 fused-step test; the z momentum is noise-sized here


def _G():
    from paper_2502_12620_amd import dgamr as G

    return G


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _workload(dim, p, N, levels):
    roots = (2, 2) if dim == 2 else (2, 2, 1)
    hi = (2.0, 2.0) if dim == 2 else (2.0, 2.0, 1.0)
    w = W.Workload(f"m{dim}{p}", dim, p, N, roots, (0.0,) * dim, hi, (0,) * dim, levels, W.IC_VORTEX,
                   [3.0, 1.0, 1.0, 0.5, 0.3, 2.0, 2.0], 1)
    if levels >= 2:
        w.initial_refinement = [lambda w_, keys: np.array([1 if k[0] == 0 else 0 for k in keys], np.int8)]
    return w


# (dim, p, N): stage workgroups of 64..256 cells, whole waves (3-D degree 3
# keeps its volume integral on the vector unit)
CASES = [(2, 2, 8), (2, 2, 16), (2, 3, 8), (2, 3, 16), (3, 2, 4), (3, 2, 8)]


@pytest.mark.parametrize("dim,p,N", CASES)
@pytest.mark.parametrize("hanging", [0, 1])
def test_mfma_residual_and_steps(dim, p, N, hanging):
    G = _G()
    print(f"mfma dim={dim} p={p} N={N} hanging={hanging}", flush=True)
    w = _workload(dim, p, N, 2)
    orc, gpu = make_pair(w, hanging=hanging, precision=G.FP32)
    rng = np.random.default_rng(dim * 100 + p * 10 + N)
    u = orc.project_ic(O.IC_VORTEX, w.ic_params)
    u[:, :, 1:, :] += 0.01 * rng.standard_normal(u[:, :, 1:, :].shape)
    g_ref = orc.fill_guards(u)
    r_ref = orc.residual(u, g_ref)
    ud, gd = _cuda(u), _cuda(g_ref)
    res = {}
    for mf in (1, 0):
        gpu.set_tuning(G.TUNE_MFMA, mf)
        rd = gpu.new_residual()
        gpu.dg_residual(ud, gd, rd)
        res[mf] = _host(rd)
        assert rel_diff(res[mf].astype(np.float64), r_ref).max() <= TOL_RES32, mf
    assert not np.array_equal(res[0], res[1])  # the matrix-core variant ran
    # fused steps
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    gpu.set_tuning(G.TUNE_MFMA, 1)
    for _ in range(3):
        orc.step(u, 0.1)
        gpu.step(ud, work, dt, 0.1)
    assert rel_diff(_host(ud), u).max() <= TOL_STATE32


def test_mfma_with_limiter_on_the_blast():
    """The blast forest at 4^3-cell blocks (degree 2, limiter): the
    matrix-core FP32 residual stays positive and near the FP64 oracle."""
    G = _G()
    w = W.sedov_c3()
    w.n_cell = 4
    orc, gpu = make_pair(w, limiter=True, precision=G.FP32)
    gpu.set_tuning(G.TUNE_MFMA, 1)
    u = orc.project_ic(O.IC_SEDOV, w.ic_params)
    ud = _cuda(u)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(4):
        orc.step(u, w.cfl, limiter=True)
        gpu.step(ud, work, dt, w.cfl)
    assert gpu.check_state(ud, work) == 0
    got = _host(ud)
    assert np.linalg.norm(got[:, 0] - u[:, 0]) / np.linalg.norm(u[:, 0]) <= 1e-5
