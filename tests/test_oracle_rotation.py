"""Pins of the oracle's rotated root frames (Sec. 3.1: neighbouring root
blocks may be rotated against each other; Sec. 3.5: the guard fill undoes
the relative rotation by an L2 projection).  A forest whose roots carry
rotated local frames describes the same physical problem as the forest with
aligned frames, so its state, mapped through the rotation (cells, modes and
momentum), must equal the aligned run.  The map is written here from the
frame definition, not taken from the oracle.  Also free stream across
rotated hanging faces, conservation, and the diffusion operator.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle as O
from tests import refmath as RM


def frame_matrix(dim, code):
    """global = Q local; 2-D: code quarter turns counter-clockwise; 3-D: the
    code-th signed permutation matrix of determinant +1 (permutations in
    lexicographic order, then sign patterns, bit l = local axis l negative)."""
    if dim == 2:
        c, s = [(1, 0), (0, 1), (-1, 0), (0, -1)][code]
        return np.array([[c, -s], [s, c]])
    out = []
    for perm in itertools.permutations(range(3)):
        for sg in range(8):
            M = np.zeros((3, 3), int)
            for l in range(3):
                M[perm[l], l] = -1 if (sg >> l) & 1 else 1
            if round(np.linalg.det(M)) == 1:
                out.append(M)
    assert len(out) == 24
    return out[code]


def to_aligned(f_rot, u_rot, frames, roots, f_al, momentum_local=True):
    """The state of the rotated forest expressed in the aligned forest's
    leaves, cells, modes and momentum components (momentum_local False:
    the rotated forest already stores the momentum along the global axes,
    as on bilinear roots)."""
    d, N, p = f_rot.dim, f_rot.N, f_rot.p
    modes = RM.graded_modes(d, p)
    R = list(roots) + [1] * (3 - d)
    al = {tuple(k): i for i, k in enumerate(f_al.keys().tolist())}
    out = np.full(f_al.state_shape(), np.nan)
    for li, (tree, level, i, j, k) in enumerate(f_rot.keys().tolist()):
        Q = frame_matrix(d, frames[tree])
        n = 2 ** (level - 1)
        loc = np.array([i, j, k][:d])
        # global leaf index inside the root: Q (loc - c) + c, c = (n - 1) / 2
        c = (n - 1) / 2.0
        glob = np.rint(Q @ (loc - c) + c).astype(int)
        key = (tree, level) + tuple(glob) + (0,) * (3 - d)
        ai = al[key]
        for cell in range(N ** d):
            cl = np.array([cell % N, (cell // N) % N, cell // (N * N)][:d])
            cg = np.rint(Q @ (cl - (N - 1) / 2.0) + (N - 1) / 2.0).astype(int)
            gcell = int(cg[0] + N * (cg[1] + (N * cg[2] if d == 3 else 0)))
            for mi, m in enumerate(modes):
                # phi_m(Q^T xi_g) = prod_l s_l^{m_l} P_{m_l}(xi_g[pi(l)])
                mg = [0, 0, 0]
                sign = 1
                for l in range(d):
                    g = int(np.flatnonzero(Q[:, l])[0])
                    mg[g] = m[l]
                    sign *= Q[g, l] ** m[l]
                gi = modes.index(tuple(mg))
                vals = u_rot[li, :, mi, cell].copy()
                if f_rot.nv == d + 2 and momentum_local:
                    vals[1:1 + d] = Q @ vals[1:1 + d]
                out[ai, :, gi, gcell] = sign * vals
    assert not np.isnan(out).any()
    return out


def _refine_tree0(f):
    fl = np.zeros(f.n_leaves, np.int8)
    fl[0] = 1
    f.adapt(fl)


@pytest.mark.parametrize("frames", [(1, 0, 0, 0), (0, 1, 2, 3), (3, 2, 1, 1)])
@pytest.mark.parametrize("p", [1, 2])
def test_2d_rotated_roots_reproduce_the_aligned_run(frames, p):
    """A 2x2 periodic root grid, root 0 refined (hanging faces on rotated
    root faces), the vortex translated for 3 steps: rotated == aligned to
    1e-13 relative, with the same time steps."""
    roots, lo, hi, prm = (2, 2), (0.0, 0.0), (10.0, 10.0), [3.0, 4.0, 6.0, 0.7, -0.4, 10.0, 10.0]
    fa = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fr = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fr.set_frames(frames)
    _refine_tree0(fa)
    _refine_tree0(fr)
    ua = fa.project_ic(O.IC_VORTEX, prm)
    ur = fr.project_ic(O.IC_VORTEX, prm)
    np.testing.assert_allclose(to_aligned(fr, ur, frames, roots, fa), ua, atol=1e-13)
    for _ in range(3):
        da = fa.step(ua, 0.1)
        dr = fr.step(ur, 0.1)
        assert dr == pytest.approx(da, rel=1e-14)
    scale = np.abs(ua).max(axis=(0, 2, 3))
    d = np.abs(to_aligned(fr, ur, frames, roots, fa) - ua).max(axis=(0, 2, 3)) / scale
    assert d.max() <= 1e-13, d
    np.testing.assert_allclose(fr.totals(ur), fa.totals(ua), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_3d_rotated_roots_reproduce_the_aligned_run(seed):
    """2x2x2 periodic roots with random frames among the 24 rotations, root
    0 refined, the vortex extruded along z (its z momentum is zero, so each
    variable's scale is floored at 1e-3 of the largest coefficient):
    rotated == aligned after 2 steps."""
    rng = np.random.default_rng(seed)
    frames = [int(x) for x in rng.integers(0, 24, 8)]
    frames[1] = 23 - frames[0]
    roots, lo, hi, prm = (2, 2, 2), (0.0,) * 3, (4.0,) * 3, [2.0, 1.5, 2.5, 0.5, 0.3, 4.0, 4.0]
    fa = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 2)
    fr = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 2)
    fr.set_frames(frames)
    _refine_tree0(fa)
    _refine_tree0(fr)
    ua = fa.project_ic(O.IC_VORTEX, prm)
    ur = fr.project_ic(O.IC_VORTEX, prm)
    for _ in range(2):
        fa.step(ua, 0.1)
        fr.step(ur, 0.1)
    big = np.abs(ua).max()
    scale = np.maximum(np.abs(ua).max(axis=(0, 2, 3)), 1e-3 * big)
    d = np.abs(to_aligned(fr, ur, frames, roots, fa) - ua).max(axis=(0, 2, 3)) / scale
    assert d.max() <= 1e-13, (frames, d)


def test_every_3d_frame_is_a_rotation_and_the_guard_fill_undoes_it():
    """Each of the 24 codes against the aligned forest: a 2-root periodic
    forest whose second root carries the code; the guard cells of the first
    root (aligned) equal those of the aligned forest (the fill undoes the
    rotation exactly: an L2 projection of a polynomial under a signed
    permutation of the axes)."""
    roots, lo, hi, prm = (2, 1, 1), (0.0,) * 3, (4.0, 2.0, 2.0), [2.0, 1.0, 1.0, 0.5, 0.3, 4.0, 2.0]
    fa = O.Forest(3, 2, 2, roots, lo, hi, (0, 0, 0), 1)
    ua = fa.project_ic(O.IC_VORTEX, prm)
    ga = fa.fill_guards(ua)
    seen = set()
    for code in range(24):
        Q = frame_matrix(3, code)
        seen.add(Q.tobytes())
        fr = O.Forest(3, 2, 2, roots, lo, hi, (0, 0, 0), 1)
        fr.set_frames([0, code])
        ur = fr.project_ic(O.IC_VORTEX, prm)
        np.testing.assert_allclose(to_aligned(fr, ur, [0, code], roots, fa), ua, atol=1e-13)
        gr = fr.fill_guards(ur)
        np.testing.assert_allclose(gr[0], ga[0], atol=1e-12)  # root 0 is aligned in both
    assert len(seen) == 24


@pytest.mark.parametrize("p", [1, 2])
def test_free_stream_across_rotated_hanging_faces(p):
    """(rho, u, v, p) = (1, 0.3, -0.2, 1) on rotated frames with hanging
    faces: the residual vanishes to round-off (the bar of the aligned
    free-stream pin: residuals carry factors 2/h up to 64 here)."""
    f = O.Forest(2, p, 4, (2, 2), (0.0, 0.0), (2.0, 2.0), (0, 0), 3)
    f.set_frames([2, 1, 3, 0])
    _refine_tree0(f)
    fl = np.zeros(f.n_leaves, np.int8)
    fl[3] = 1
    f.adapt(fl)
    u = f.project_ic(O.IC_UNIFORM, [1.0, 0.3, -0.2, 0.0, 1.0])
    r = f.residual(u)
    assert np.abs(r).max() < 1e-11


def test_conservation_on_a_conforming_rotated_forest():
    f = O.Forest(2, 2, 4, (2, 2), (0.0, 0.0), (10.0, 10.0), (0, 0), 1)
    f.set_frames([0, 3, 1, 2])
    u = f.project_ic(O.IC_VORTEX, [3.0, 4.0, 6.0, 0.7, -0.4, 10.0, 10.0])
    t0 = f.totals(u)
    for _ in range(5):
        f.step(u, 0.1)
    np.testing.assert_allclose(f.totals(u), t0, rtol=1e-13, atol=1e-13)


def test_diffusion_on_rotated_roots():
    """The diffusion operator is isotropic: rotated frames reproduce the
    aligned run of Sec. 5.2's exact solution, Dirichlet faces included."""
    roots, lo, hi = (2, 2), (0.0, 0.0), (1.0, 1.0)
    kw = dict(equation=O.EQ_DIFFUSION, nu=1.0, avec=(-1.0, 1.0))
    fa = O.Forest(2, 2, 4, roots, lo, hi, (2, 2), 2, **kw)
    fr = O.Forest(2, 2, 4, roots, lo, hi, (2, 2), 2, **kw)
    frames = [1, 2, 3, 1]
    fr.set_frames(frames)
    _refine_tree0(fa)
    _refine_tree0(fr)
    ua = fa.project_ic(O.IC_EXP, [])
    ur = fr.project_ic(O.IC_EXP, [])
    for _ in range(5):
        fa.step(ua, 0.006)
        fr.step(ur, 0.006)
    d = np.abs(to_aligned(fr, ur, frames, roots, fa) - ua).max() / np.abs(ua).max()
    assert d <= 1e-13


def test_frames_are_refused_where_they_are_not_defined():
    f = O.Forest(2, 1, 4, (2, 1), (0.0, 0.0), (2.0, 2.0), (0, 0), 1)  # 1 x 2 root edges
    with pytest.raises(ValueError):
        f.set_frames([1, 0])
    g = O.Forest(2, 1, 4, (2, 2), (0.0, 0.0), (2.0, 2.0), (0, 0), 1, hanging=O.HANG_CONSERVATIVE)
    with pytest.raises(ValueError):
        g.set_frames([1, 0, 0, 0])
    h = O.Forest(2, 1, 4, (2, 2), (0.0, 0.0), (2.0, 2.0), (0, 0), 1)
    with pytest.raises(ValueError):
        h.set_frames([4, 0, 0, 0])


@pytest.mark.parametrize("frames", [(1, 0, 0, 0), (0, 3, 2, 1)])
@pytest.mark.parametrize("p", [1, 2])
def test_2d_convection_on_rotated_roots_reproduces_the_aligned_run(frames, p):
    """Scalar convection (Sec. 5.1) with the velocity taken along each
    root's local axes, root 0 refined: rotated == aligned after 4 steps
    (cells and modes mapped through the frames; one scalar variable)."""
    roots, lo, hi, vel = (2, 2), (0.0, 0.0), (1.0, 1.0), (1.0, 0.5, 0.0)
    kw = dict(equation=O.EQ_ADVECTION, velocity=vel)
    fa = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2, **kw)
    fr = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2, **kw)
    fr.set_frames(frames)
    _refine_tree0(fa)
    _refine_tree0(fr)
    prm = [1.0, 1.0, 1.0, 1.0]
    ua = fa.project_ic(O.IC_COSINE, prm)
    ur = fr.project_ic(O.IC_COSINE, prm)
    np.testing.assert_allclose(to_aligned(fr, ur, frames, roots, fa), ua, atol=1e-14)
    for _ in range(4):
        assert fr.step(ur, 0.2) == pytest.approx(fa.step(ua, 0.2), rel=1e-14)
    assert np.abs(to_aligned(fr, ur, frames, roots, fa) - ua).max() <= 1e-13 * np.abs(ua).max()
    np.testing.assert_allclose(fr.totals(ur), fa.totals(ua), rtol=1e-13, atol=1e-14)


def test_3d_convection_on_rotated_roots_reproduces_the_aligned_run():
    frames = (5, 17, 0, 9, 12, 3, 23, 1)
    roots, lo, hi, vel = (2, 2, 2), (0.0,) * 3, (1.0,) * 3, (1.0, 0.5, 0.25)
    kw = dict(equation=O.EQ_ADVECTION, velocity=vel)
    fa = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 2, **kw)
    fr = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 2, **kw)
    fr.set_frames(frames)
    _refine_tree0(fa)
    _refine_tree0(fr)
    prm = [1.0, 1.0, 1.0, 1.0]
    ua = fa.project_ic(O.IC_COSINE, prm)
    ur = fr.project_ic(O.IC_COSINE, prm)
    for _ in range(3):
        assert fr.step(ur, 0.2) == pytest.approx(fa.step(ua, 0.2), rel=1e-14)
    assert np.abs(to_aligned(fr, ur, frames, roots, fa) - ua).max() <= 1e-13 * np.abs(ua).max()
