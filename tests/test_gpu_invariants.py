"""Invariants of the GPU step at any size, for every stage kernel: a uniform
state stays uniform across refinement interfaces (free-stream
preservation, both hanging modes), and the conservative hanging mode keeps
the discrete totals of all conserved variables to round-off on a forest
with coarse-fine faces."""
import numpy as np
import pytest

from paper_2502_12620_amd import workloads as W
from tests.gpu_helpers import make_pair
from tests.test_gpu_parity import _cuda, _forest, _host, _physical_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (dim, stage kernel variant): 2-D lane per (cell, variable) and thread per
# cell; 3-D lane per (cell, variable) (paper hanging mode only) and thread
# per cell
KERNELS = [(2, 0), (2, 1), (3, 0), (3, 1)]


def _run(gpu, ud, variant, steps, cfl=0.2):
    from paper_2502_12620_amd import dgamr as G

    gpu.set_tuning(G.TUNE_STAGE_VARIANT, variant)
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        gpu.step(ud, work, dt, cfl)
    return work


@pytest.mark.parametrize("dim,variant", KERNELS)
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("hanging", [0, 1])
def test_free_stream_across_refinement(dim, variant, p, hanging):
    from paper_2502_12620_amd import dgamr as G

    w = _forest(dim, p, 4, 3)
    orc, gpu = make_pair(w, hanging=hanging)
    # rho, u, v, w (3-D), p
    ud = gpu.project_ic(G.IC_UNIFORM, [1.2, 0.3, -0.2, 0.1, 2.5])
    u0 = _host(ud).copy()
    _run(gpu, ud, variant, 3)
    got = _host(ud)
    assert np.abs(got - u0).max() <= 1e-13 * np.abs(u0).max()


@pytest.mark.parametrize("dim,variant", KERNELS)
@pytest.mark.parametrize("p", [1, 2])
def test_conservative_mode_conserves_every_variable(dim, variant, p):
    """(The 3-D lane kernel does not take mortar faces: variant 0 runs one
    thread per cell there, which this checks as well.)"""
    w = _forest(dim, p, 4, 3, bc=W.PERIODIC)
    orc, gpu = make_pair(w, hanging=1)
    ud = _cuda(_physical_state(orc, w, seed=70 + p))
    work = gpu.new_work()
    t0 = _host(gpu.conserved_totals(ud, work)).copy()
    work = _run(gpu, ud, variant, 5)
    t1 = _host(gpu.conserved_totals(ud, work))
    scale = np.abs(t0).max()
    assert np.abs(t1 - t0).max() <= 1e-13 * scale, (t0, t1)
