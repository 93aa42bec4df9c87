"""Seeded random forests against the oracle.  Each case draws the
dimension, degree, block size, root grid, boundary kinds, the equation
(Euler or scalar convection), hanging mode, rotated root frames, distorted
root nodes and the positivity limiter
(within what each feature supports), refines twice by random flags, and then
compares the initial projection and three fused steps (time steps, states,
conserved totals) with the oracle.  FP64 bar 1e-12 relative per variable.
The draw is printed before each case."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import rel_diff_floored
from tests.test_oracle_mapped import distorted_nodes, distorted_nodes3

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _draw(seed):
    rng = np.random.default_rng(7000 + seed)
    dim = 2 if rng.random() < 0.6 else 3
    p = int(rng.integers(1, 4)) if dim == 2 else int(rng.integers(1, 3))
    N = int(rng.choice([2, 4, 6])) if dim == 2 else int(rng.choice([2, 4]))
    roots = tuple(int(x) for x in rng.integers(1, 4, dim)) if dim == 2 else tuple(int(x) for x in rng.integers(1, 3, 3))
    h = 2.5
    lo = tuple(0.0 for _ in range(dim))
    hi = tuple(h * r for r in roots)
    bc = tuple(int(x) for x in rng.integers(0, 2, dim))
    mapped = bool(rng.random() < 0.4)
    frames = bool(rng.random() < 0.4)
    conservative = (not mapped) and (not frames) and bool(rng.random() < 0.3)
    advection = bool(rng.random() < 0.25)
    limiter = (not advection) and bool(rng.random() < 0.3)
    return dict(dim=dim, p=p, N=N, roots=roots, lo=lo, hi=hi, bc=bc, mapped=mapped, frames=frames,
                conservative=conservative, advection=advection, limiter=limiter, rng=rng)


@pytest.mark.parametrize("seed", range(48))
def test_random_forest_matches_the_oracle(seed):
    from paper_2502_12620_amd import dgamr as G

    c = _draw(seed)
    rng = c.pop("rng")
    print(f"random forest {seed}: {c}", flush=True)
    dim, p, N, roots, lo, hi, bc = c["dim"], c["p"], c["N"], c["roots"], c["lo"], c["hi"], c["bc"]
    hang = 1 if c["conservative"] else 0
    vel = (1.0, 0.5, 0.25)
    kw_o = dict(equation=O.EQ_ADVECTION, velocity=vel) if c["advection"] else {}
    kw_g = dict(equation=G.EQ_ADVECTION, velocity=vel) if c["advection"] else {}
    orc = O.Forest(dim, p, N, roots, lo, hi, bc, 3, hanging=hang, **kw_o)
    gpu = G.Forest(dim, p, N, roots, lo, hi, bc, 3, hanging=hang,
                   limiter=G.LIMITER_POSITIVITY if c["limiter"] else G.LIMITER_NONE, **kw_g)
    if c["frames"]:
        codes = [int(x) for x in rng.integers(0, 4 if dim == 2 else 24, int(np.prod(roots)))]
        orc.set_frames(codes)
        gpu.set_root_frames(codes)
    if c["mapped"]:
        nodes = (distorted_nodes(roots, lo, hi, 0.15, seed=seed) if dim == 2
                 else distorted_nodes3(roots, lo, hi, 0.12, seed=seed))
        orc.set_nodes(nodes)
        gpu.set_root_nodes(nodes)
    for _ in range(2):
        flags = (rng.random(orc.n_leaves) < 0.35).astype(np.int8)
        orc.adapt(flags)
        gpu.adapt(flags, torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))
    assert np.array_equal(orc.keys(), gpu.keys())
    # the vortex centre off every quadrature node (its periodic seam too)
    L = [hi[a] - lo[a] for a in range(dim)]
    if c["advection"]:
        kind_o, kind_g, prm = O.IC_COSINE, G.IC_COSINE, [1.0] + L
    else:
        kind_o, kind_g, prm = O.IC_VORTEX, G.IC_VORTEX, [3.0, 0.4137 * L[0], 0.5821 * L[1], 0.5, 0.3, L[0], L[1]]
    u = orc.project_ic(kind_o, prm)
    ud = gpu.project_ic(kind_g, prm)
    assert rel_diff_floored(ud.cpu().numpy(), u, 1e-3).max() <= TOL
    work, dt = gpu.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dref = orc.step(u, 0.1, limiter=c["limiter"])
        gpu.step(ud, work, dt, 0.1)
        torch.cuda.synchronize()
        assert dt.cpu().numpy()[0] == pytest.approx(dref, rel=1e-13)
    assert rel_diff_floored(ud.cpu().numpy(), u, 1e-3).max() <= TOL
    tot = gpu.conserved_totals(ud, work).cpu().numpy()
    np.testing.assert_allclose(tot, orc.totals(u), rtol=1e-12, atol=1e-12 * np.abs(orc.totals(u)).max())
    assert gpu.check_state(ud, work) == 0
