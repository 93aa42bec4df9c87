"""The allocation-free step (dgamr_step_static, a static device work area)
against dgamr_step with a caller-owned work buffer: the same launches, so
the states and time steps must agree bit for bit, on two calls in a row
with a smaller forest the second time, in 3-D where the work area also
holds the guard traces of the lane kernel, and on rotated and bilinear roots
whose stages fill its guard buffer."""
import numpy as np
import pytest

from paper_2502_12620_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _forest(G, w, setup=None, limiter=False):
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                 limiter=G.LIMITER_POSITIVITY if limiter else G.LIMITER_NONE)
    if setup is not None:
        setup(f)
    z = torch.zeros(f.state_shape(), dtype=torch.float64, device="cuda")
    for rule in w.initial_refinement:
        z = f.adapt(rule(w, f.keys()), z)
    return f


def _compare(G, w, steps, setup=None, limiter=False):
    f = _forest(G, w, setup, limiter)
    print(f"static step: {w.name}, {f.n_leaves} leaves, {steps} steps", flush=True)
    u0 = f.project_ic(G.IC_VORTEX, w.ic_params)
    ua, ub = u0.clone(), u0.clone()
    work = f.new_work()
    dta = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        f.step(ua, work, dta, w.cfl)
        f.step_static(ub, dtb, w.cfl)
    torch.cuda.synchronize()
    assert torch.equal(ua, ub)
    assert torch.equal(dta, dtb)
    assert torch.isfinite(ub).all()


def test_static_step_equals_step_on_two_calls_in_a_row():
    from paper_2502_12620_amd import dgamr as G

    _compare(G, W.vortex_c2(), 3)   # 100 leaves of 16^2 cells, degree 2
    _compare(G, W.vortex_c1(), 3)   # then a smaller forest: 16 leaves of 8^2 cells


def test_static_step_in_3d_with_guard_traces():
    from paper_2502_12620_amd import dgamr as G

    w = W.roofline_3d(2, 3)   # degree 3: the lane kernel reads guard traces from the work area
    w.n_cell = 4
    _compare(G, w, 2)
    _compare(G, W.vortex_c1(), 2)


@pytest.mark.parametrize("roots", ["rotated", "mapped", "mapped_limited"])
def test_static_step_on_rotated_and_bilinear_roots(roots):
    """Forests whose stages first fill the guard buffer of the work area:
    a rotated frame on every root, or bilinear roots (also with the
    positivity limiter); then a plain forest."""
    from paper_2502_12620_amd import dgamr as G

    w = W.roofline_2d(4, 2)
    w.n_cell = 8
    if roots == "rotated":
        frames = W.random_root_frames(w)
        _compare(G, w, 2, lambda f: f.set_root_frames(frames))
    else:
        nodes = W.smooth_root_nodes(w)
        _compare(G, w, 2, lambda f: f.set_root_nodes(nodes), limiter=roots == "mapped_limited")
    _compare(G, W.vortex_c1(), 2)


def test_static_step_refuses_a_forest_above_the_static_size():
    from paper_2502_12620_amd import dgamr as G

    w = W.roofline_2d(32, 2)  # 1024 leaves of 16^2 cells: a 50 MB state, ~190 MB + guards of work
    w.roots = (48, 48)
    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma)
    assert f.sizes()[3] > (256 << 20)
    u = f.new_state()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(G.DgamrError) as e:
        f.step_static(u, dt)
    assert e.value.code == G.EUNSUPPORTED
