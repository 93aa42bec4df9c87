"""Pins of the oracle's bilinear root blocks (Sec. 3.3, Eq. 6: a root is the
bilinear image of the reference square spanned by its corner nodes; the
weak form of Eq. 3-4 then carries the map's Jacobian at every point and the
full mass matrix).  The pins come from outside that code: rectangular nodes
reproduce the axis-aligned oracle; a uniform state stays a steady solution
on distorted roots with hanging faces (the discrete metric identities of a
bilinear map); conforming distorted forests conserve every variable (Euler and scalar
convection); the isentropic vortex converges at order p+1 on a smoothly
distorted periodic grid; folded roots and unmatched periodic nodes are
refused.  With rotated root frames: rectangular nodes reproduce the aligned
box grid once the frames' cell and mode permutation is undone (the momentum
stays along the global axes), and on distorted roots the choice of frames
does not change the solution.  CPU only."""
import numpy as np
import pytest

import oracle as O

PRM = [3.0, 5.0, 5.0, 0.7, -0.4, 10.0, 10.0]


def box_nodes(roots, lo, hi):
    nx, ny = roots
    g = np.zeros((ny + 1, nx + 1, 2))
    g[..., 0] = np.linspace(lo[0], hi[0], nx + 1)[None, :]
    g[..., 1] = np.linspace(lo[1], hi[1], ny + 1)[:, None]
    return g


def distorted_nodes(roots, lo, hi, amp, seed=0):
    """Box nodes with the interior nodes and, periodically, the boundary
    nodes moved by up to amp of a root edge (opposite boundaries move
    together, so the grid stays periodic)."""
    g = box_nodes(roots, lo, hi)
    nx, ny = roots
    h = min((hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny)
    rng = np.random.default_rng(seed)
    d = amp * h * rng.uniform(-1, 1, (ny, nx, 2))
    for j in range(ny + 1):
        for i in range(nx + 1):
            g[j, i] += d[j % ny, i % nx]
    return g


def smooth_nodes(roots, lo, hi, amp):
    """x + amp sin(2 pi x/L) sin(2 pi y/L) style periodic distortion."""
    g = box_nodes(roots, lo, hi)
    L = np.array(hi) - np.array(lo)
    x, y = g[..., 0].copy(), g[..., 1].copy()
    s = np.sin(2 * np.pi * (x - lo[0]) / L[0]) * np.sin(2 * np.pi * (y - lo[1]) / L[1])
    g[..., 0] = x + amp * L[0] * s
    g[..., 1] = y + amp * L[1] * s
    return g


def _refine(f, which):
    fl = np.zeros(f.n_leaves, np.int8)
    fl[which] = 1
    f.adapt(fl)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rectangular_nodes_reproduce_the_box_grid(p):
    roots, lo, hi = (2, 2), (0.0, 0.0), (10.0, 10.0)
    fa = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fm = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fm.set_nodes(box_nodes(roots, lo, hi))
    for f in (fa, fm):
        _refine(f, 0)
    ua, um = fa.project_ic(O.IC_VORTEX, PRM), fm.project_ic(O.IC_VORTEX, PRM)
    np.testing.assert_allclose(um, ua, atol=1e-14)
    for _ in range(3):
        assert fm.step(um, 0.1) == pytest.approx(fa.step(ua, 0.1), rel=1e-14)
    assert np.abs(um - ua).max() <= 1e-13 * np.abs(ua).max()
    np.testing.assert_allclose(fm.totals(um), fa.totals(ua), rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("bc", [0, 1])
def test_free_stream_on_distorted_roots_with_hanging_faces(p, bc):
    roots, lo, hi = (3, 3), (0.0, 0.0), (3.0, 3.0)
    f = O.Forest(2, p, 4, roots, lo, hi, (bc, bc), 3)
    f.set_nodes(distorted_nodes(roots, lo, hi, 0.2, seed=p))
    _refine(f, 4)
    _refine(f, 0)
    u = f.project_ic(O.IC_UNIFORM, [1.0, 0.3, -0.2, 0.0, 1.0])
    assert np.abs(u[:, :, 1:]).max() < 1e-13  # the projection of a constant is the constant
    assert np.abs(f.residual(u)).max() < 1e-11


@pytest.mark.parametrize("p", [1, 2])
def test_conservation_on_distorted_conforming_roots(p):
    roots, lo, hi = (3, 2), (0.0, 0.0), (10.0, 10.0)
    f = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 1)
    f.set_nodes(distorted_nodes(roots, lo, hi, 0.25, seed=7))
    u = f.project_ic(O.IC_VORTEX, PRM)
    t0 = f.totals(u)
    for _ in range(5):
        f.step(u, 0.1)
    np.testing.assert_allclose(f.totals(u), t0, rtol=1e-13, atol=1e-12)


def test_advection_conservation_and_positivity_of_the_map():
    roots, lo, hi = (2, 2), (0.0, 0.0), (1.0, 1.0)
    f = O.Forest(2, 2, 4, roots, lo, hi, (0, 0), 1, equation=O.EQ_ADVECTION, velocity=(1.0, 0.5, 0.0))
    f.set_nodes(distorted_nodes(roots, lo, hi, 0.2, seed=3))
    u = f.project_ic(O.IC_COSINE, [1.0, 1.0, 1.0, 1.0])
    t0 = f.totals(u)
    for _ in range(5):
        f.step(u, 0.1)
    np.testing.assert_allclose(f.totals(u), t0, rtol=1e-13, atol=1e-13)
    bad = box_nodes(roots, lo, hi)
    bad[1, 1] = [1.2, 1.2]  # folds the four roots around the centre node
    g = O.Forest(2, 2, 4, roots, lo, hi, (0, 0), 1)
    with pytest.raises(ValueError):
        g.set_nodes(bad)
    moved = box_nodes(roots, lo, hi)
    moved[0, 2, 1] += 0.01  # the periodic copy of node (0, 0) no longer matches
    with pytest.raises(ValueError):
        g.set_nodes(moved)


@pytest.mark.parametrize("p", [1, 2])
def test_vortex_order_on_a_smoothly_distorted_grid(p):
    """L2 density error against the exact translated vortex on 4x4 roots of
    N = 8 and 16 cells, periodic [0, 20]^2 (the periodic kink negligible),
    nodes moved by a smooth periodic field: observed order >= p + 1 - 0.2,
    the bar of the box-grid order pins."""
    lo, hi, roots = (0.0, 0.0), (20.0, 20.0), (4, 4)
    prm = [5.0, 10.0, 10.0, 1.0, 1.0, 20.0, 20.0]
    T = 0.5
    errs = []
    for N in (8, 16):
        f = O.Forest(2, p, N, roots, lo, hi, (0, 0), 1)
        f.set_nodes(smooth_nodes(roots, lo, hi, 0.03))
        u = f.project_ic(O.IC_VORTEX, prm)
        h = 20.0 / (4 * N)
        dt = 0.05 * h
        n = int(round(T / dt))
        for _ in range(n):
            f.step(u, dt=T / n)
        l1, l2 = f.errors(u, O.IC_VORTEX, prm, T)
        errs.append(l2[0])
    order = np.log2(errs[0] / errs[1])
    assert order >= p + 1 - 0.2, (errs, order)


def box_nodes3(roots, lo, hi):
    nx, ny, nz = roots
    g = np.zeros((nz + 1, ny + 1, nx + 1, 3))
    g[..., 0] = np.linspace(lo[0], hi[0], nx + 1)[None, None, :]
    g[..., 1] = np.linspace(lo[1], hi[1], ny + 1)[None, :, None]
    g[..., 2] = np.linspace(lo[2], hi[2], nz + 1)[:, None, None]
    return g


def distorted_nodes3(roots, lo, hi, amp, seed=0):
    """3-D box nodes moved by up to amp of a root edge, periodically."""
    g = box_nodes3(roots, lo, hi)
    nx, ny, nz = roots
    h = min((hi[a] - lo[a]) / roots[a] for a in range(3))
    rng = np.random.default_rng(seed)
    d = amp * h * rng.uniform(-1, 1, (nz, ny, nx, 3))
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                g[k, j, i] += d[k % nz, j % ny, i % nx]
    return g


PRM3 = [2.0, 1.3, 2.7, 0.5, 0.3, 4.0, 4.0]  # the periodic seam of the vortex off every Gauss node


@pytest.mark.parametrize("p", [1, 2])
def test_3d_box_nodes_reproduce_the_box_grid(p):
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (4.0,) * 3
    fa = O.Forest(3, p, 2, roots, lo, hi, (0, 0, 0), 2)
    fm = O.Forest(3, p, 2, roots, lo, hi, (0, 0, 0), 2)
    fm.set_nodes(box_nodes3(roots, lo, hi))
    for f in (fa, fm):
        _refine(f, 0)
    ua, um = fa.project_ic(O.IC_VORTEX, PRM3), fm.project_ic(O.IC_VORTEX, PRM3)
    np.testing.assert_allclose(um, ua, atol=1e-14)
    for _ in range(2):
        assert fm.step(um, 0.1) == pytest.approx(fa.step(ua, 0.1), rel=1e-14)
    assert np.abs(um - ua).max() <= 1e-13 * np.abs(ua).max()


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("bc", [0, 1])
def test_3d_free_stream_on_distorted_roots_with_hanging_faces(p, bc):
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (2.0,) * 3
    f = O.Forest(3, p, 2, roots, lo, hi, (bc,) * 3, 3)
    f.set_nodes(distorted_nodes3(roots, lo, hi, 0.15, seed=p + 3 * bc))
    _refine(f, 0)
    _refine(f, 1)
    u = f.project_ic(O.IC_UNIFORM, [1.0, 0.3, -0.2, 0.1, 1.0])
    assert np.abs(u[:, :, 1:]).max() < 1e-13
    assert np.abs(f.residual(u)).max() < 1e-11


def test_3d_conservation_on_distorted_conforming_roots():
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (4.0,) * 3
    f = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 1)
    f.set_nodes(distorted_nodes3(roots, lo, hi, 0.2, seed=5))
    u = f.project_ic(O.IC_VORTEX, PRM3)
    t0 = f.totals(u)
    for _ in range(3):
        f.step(u, 0.1)
    np.testing.assert_allclose(f.totals(u), t0, rtol=1e-13, atol=1e-12)


def test_3d_folded_root_is_refused():
    roots, lo, hi = (2, 2, 2), (0.0,) * 3, (2.0,) * 3
    g = box_nodes3(roots, lo, hi)
    g[1, 1, 1] = [1.9, 1.9, 1.9]  # the centre node pushed through the far corner
    f = O.Forest(3, 1, 2, roots, lo, hi, (1, 1, 1), 1)
    with pytest.raises(ValueError):
        f.set_nodes(g)


# ---------------------------------------------------------------- rotated frames on bilinear / trilinear roots

from tests.test_oracle_rotation import to_aligned  # noqa: E402


def _refine_tree0(f):
    fl = np.zeros(f.n_leaves, np.int8)
    fl[0] = 1
    f.adapt(fl)


@pytest.mark.parametrize("frames", [(1, 0, 0, 0), (0, 1, 2, 3), (3, 2, 1, 1)])
@pytest.mark.parametrize("p", [1, 2])
def test_rectangular_nodes_with_frames_reproduce_the_aligned_box_grid(frames, p):
    """Rotated frames and rectangular nodes, root 0 refined (hanging faces on
    rotated faces): after three steps the state, with the frames' cell and
    mode permutation undone, equals the aligned box-grid run."""
    roots, lo, hi = (2, 2), (0.0, 0.0), (10.0, 10.0)
    fa = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fm = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fm.set_frames(frames)
    fm.set_nodes(box_nodes(roots, lo, hi))
    _refine_tree0(fa)
    _refine_tree0(fm)
    ua, um = fa.project_ic(O.IC_VORTEX, PRM), fm.project_ic(O.IC_VORTEX, PRM)
    np.testing.assert_allclose(to_aligned(fm, um, frames, roots, fa, momentum_local=False), ua, atol=1e-13)
    for _ in range(3):
        assert fm.step(um, 0.1) == pytest.approx(fa.step(ua, 0.1), rel=1e-13)
    got = to_aligned(fm, um, frames, roots, fa, momentum_local=False)
    assert np.abs(got - ua).max() <= 1e-12 * np.abs(ua).max()
    np.testing.assert_allclose(fm.totals(um), fa.totals(ua), rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("p", [1, 2])
def test_frames_do_not_change_the_solution_on_distorted_roots(p):
    """The same distorted periodic root grid with and without rotated
    frames, root 0 refined: the same physical solution after three steps."""
    roots, lo, hi, frames = (2, 2), (0.0, 0.0), (10.0, 10.0), (2, 1, 3, 1)
    nodes = distorted_nodes(roots, lo, hi, 0.2, seed=11)
    fa = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fm = O.Forest(2, p, 4, roots, lo, hi, (0, 0), 2)
    fa.set_nodes(nodes)
    fm.set_nodes(nodes)
    fm.set_frames(frames)  # after the nodes: either order
    _refine_tree0(fa)
    _refine_tree0(fm)
    ua, um = fa.project_ic(O.IC_VORTEX, PRM), fm.project_ic(O.IC_VORTEX, PRM)
    np.testing.assert_allclose(to_aligned(fm, um, frames, roots, fa, momentum_local=False), ua,
                               atol=1e-12 * np.abs(ua).max())
    for _ in range(3):
        assert fm.step(um, 0.1) == pytest.approx(fa.step(ua, 0.1), rel=1e-12)
    got = to_aligned(fm, um, frames, roots, fa, momentum_local=False)
    assert np.abs(got - ua).max() <= 1e-11 * np.abs(ua).max()


@pytest.mark.parametrize("bc", [0, 1])
def test_free_stream_on_rotated_distorted_roots_with_hanging_faces(bc):
    roots, lo, hi = (3, 3), (0.0, 0.0), (3.0, 3.0)
    f = O.Forest(2, 2, 4, roots, lo, hi, (bc, bc), 3)
    f.set_frames([1, 0, 3, 2, 1, 0, 0, 2, 3])
    f.set_nodes(distorted_nodes(roots, lo, hi, 0.2, seed=5))
    _refine(f, 4)
    _refine(f, 0)
    u = f.project_ic(O.IC_UNIFORM, [1.0, 0.3, -0.2, 0.0, 1.0])
    assert np.abs(f.residual(u)).max() < 1e-11


def test_3d_box_nodes_with_frames_reproduce_the_aligned_box_grid():
    roots, lo, hi, frames = (2, 2, 2), (0.0,) * 3, (4.0,) * 3, (5, 0, 17, 9, 0, 23, 2, 12)
    fa = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 2)
    fm = O.Forest(3, 1, 2, roots, lo, hi, (0, 0, 0), 2)
    fm.set_frames(frames)
    fm.set_nodes(box_nodes3(roots, lo, hi))
    _refine_tree0(fa)
    _refine_tree0(fm)
    ua, um = fa.project_ic(O.IC_VORTEX, PRM3), fm.project_ic(O.IC_VORTEX, PRM3)
    np.testing.assert_allclose(to_aligned(fm, um, frames, roots, fa, momentum_local=False), ua, atol=1e-13)
    for _ in range(2):
        assert fm.step(um, 0.1) == pytest.approx(fa.step(ua, 0.1), rel=1e-13)
    got = to_aligned(fm, um, frames, roots, fa, momentum_local=False)
    assert np.abs(got - ua).max() <= 1e-12 * np.abs(ua).max()


# ------------------------------------------------------------------ positivity limiter
def _limiter_points(p):
    """Zhang-Shu points of the 2-D tensor cell (Lobatto along one axis with
    the fewest points exact for degree p, Gauss along the other) and the
    volume Gauss points."""
    from tests import refmath as RM

    L = 2
    while 2 * L - 3 < p:
        L += 1
    lob = {2: [-1.0, 1.0], 3: [-1.0, 0.0, 1.0], 4: [-1.0, -5 ** -0.5, 5 ** -0.5, 1.0]}[L]
    xg, _ = np.polynomial.legendre.leggauss(p + 1)
    vol, _ = RM.tensor_gauss(2, p + 1)
    pts = [tuple(x) for x in vol] + [(a, b) for a in lob for b in xg] + [(b, a) for a in lob for b in xg]
    return np.array(pts)


def _physical_means(u, nodes, p, N):
    """Cell means over the physical cells of a single unrefined bilinear
    root, int U |J| / int |J| with a 6-point Gauss rule per axis (the
    test's own map: X(s) = sum of the corner nodes times the bilinear
    weights of s in [0,1]^2; cell (i, j) covers s in [i/N,(i+1)/N] x
    [j/N,(j+1)/N], cell index i + N j)."""
    from tests import refmath as RM

    modes = RM.graded_modes(2, p)
    xi, w = RM.tensor_gauss(2, 6)
    X = nodes  # X[y][x] = node (x, y)
    out = np.zeros((N * N, u.shape[1]))
    for c in range(N * N):
        ci, cj = c % N, c // N
        s0 = (ci + 0.5 * (xi[:, 0] + 1.0)) / N
        s1 = (cj + 0.5 * (xi[:, 1] + 1.0)) / N
        dx_ds0 = (1 - s1)[:, None] * (X[0, 1] - X[0, 0]) + s1[:, None] * (X[1, 1] - X[1, 0])
        dx_ds1 = (1 - s0)[:, None] * (X[1, 0] - X[0, 0]) + s0[:, None] * (X[1, 1] - X[0, 1])
        det = dx_ds0[:, 0] * dx_ds1[:, 1] - dx_ds0[:, 1] * dx_ds1[:, 0]
        assert det.min() > 0
        vals = RM.eval_cell(u[0, :, :, c], modes, xi)
        out[c] = (w * det) @ vals / np.sum(w * det)
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_limiter_keeps_each_physical_cell_mean_on_a_bilinear_root(p):
    """On a distorted root the cell mean is the one over the physical cell,
    not mode 0: the limiter must keep that mean in every cell (a limiter
    scaling about mode 0 moves it), and leave density and pressure >= eps
    at the Zhang-Shu points."""
    from tests import refmath as RM

    N = 4
    nodes = np.array([[[0.0, 0.0], [1.0, 0.15]], [[0.25, 0.9], [1.4, 1.3]]])
    f = O.Forest(2, p, N, (1, 1), (0.0, 0.0), (1.0, 1.0), (1, 1), 1)
    f.set_nodes(nodes)
    u = f.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1.0])
    rng = np.random.default_rng(40 + p)
    u[0, :, 1:, :] = 0.6 * rng.standard_normal(u[0, :, 1:, :].shape)  # wild higher modes
    before = u.copy()
    m0 = _physical_means(u, nodes, p, N)
    assert m0[:, 0].min() > 0.2
    assert np.abs(m0 - before[0, :, 0, :].T).max() > 1e-3  # the physical mean is not mode 0
    f.limit(u)
    m1 = _physical_means(u, nodes, p, N)
    np.testing.assert_allclose(m1, m0, rtol=1e-13, atol=1e-13)
    assert np.abs(u[0, :, 0, :] - before[0, :, 0, :]).max() > 1e-6  # mode 0 moved
    vals = np.stack([RM.eval_cell(u[0, :, :, c], RM.graded_modes(2, p), _limiter_points(p)) for c in range(N * N)])
    rho, _, pr = RM.euler_primitives(vals, 2, 1.4)
    assert rho.min() >= 1e-13 - 1e-14 and pr.min() >= 1e-13 - 1e-14


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (3, 1)])
def test_limited_steps_on_box_nodes_match_the_box_grid(dim, p):
    """With rectangular nodes the physical mean is mode 0 and the limited
    steps are the box grid's (Zhang-Shu on tensor cells)."""
    if dim == 2:
        roots, lo, hi, nodes = (2, 2), (0.0, 0.0), (4.0, 4.0), box_nodes((2, 2), (0.0, 0.0), (4.0, 4.0))
    else:
        roots, lo, hi = (2, 2, 2), (0.0,) * 3, (4.0,) * 3
        nodes = box_nodes3(roots, lo, hi)
    fa = O.Forest(dim, p, 4 if dim == 2 else 2, roots, lo, hi, (1,) * dim, 2)
    fm = O.Forest(dim, p, 4 if dim == 2 else 2, roots, lo, hi, (1,) * dim, 2)
    fm.set_nodes(nodes)
    for f in (fa, fm):
        _refine(f, 0)
    ua = fa.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1e-3])
    ua[0, dim + 1, 0, :] = 1e3 / 0.4
    um = ua.copy()
    for _ in range(3):
        assert fm.step(um, 0.1, limiter=True) == pytest.approx(fa.step(ua, 0.1, limiter=True), rel=1e-13)
    assert np.abs(um - ua).max() <= 1e-12 * np.abs(ua).max()
    t = fm.totals(um)
    np.testing.assert_allclose(t, fa.totals(ua), rtol=1e-12, atol=1e-12 * np.abs(t).max())


def _physical_means3(u, nodes, p, N):
    """The same on a single unrefined trilinear root: X(s) = sum over the
    corners b in {0,1}^3 of prod_a (s_a or 1 - s_a) times the node; cell
    (i, j, k) covers s in [i/N,(i+1)/N] x [j/N,(j+1)/N] x [k/N,(k+1)/N],
    cell index i + N (j + N k); |J| from the three columns dX/ds_a."""
    from tests import refmath as RM

    modes = RM.graded_modes(3, p)
    xi, w = RM.tensor_gauss(3, 5)
    out = np.zeros((N ** 3, u.shape[1]))
    for c in range(N ** 3):
        ijk = (c % N, (c // N) % N, c // (N * N))
        s = np.stack([(ijk[a] + 0.5 * (xi[:, a] + 1.0)) / N for a in range(3)], axis=-1)
        J = np.zeros((len(w), 3, 3))
        for b in range(8):
            bits = [(b >> a) & 1 for a in range(3)]
            X = nodes[bits[2], bits[1], bits[0]]
            fac = [s[:, a] if bits[a] else 1.0 - s[:, a] for a in range(3)]
            for a in range(3):
                d = (1.0 if bits[a] else -1.0) * np.prod([fac[e] for e in range(3) if e != a], axis=0)
                J[:, :, a] += d[:, None] * X[None, :]
        det = np.linalg.det(J)
        assert det.min() > 0
        vals = RM.eval_cell(u[0, :, :, c], modes, xi)
        out[c] = (w * det) @ vals / np.sum(w * det)
    return out


@pytest.mark.parametrize("p", [1, 2])
def test_limiter_keeps_each_physical_cell_mean_on_a_trilinear_root(p):
    """3-D: the limiter keeps every cell's mean over the physical cell of a
    distorted trilinear root and moves mode 0."""
    N = 2
    nodes = np.zeros((2, 2, 2, 3))  # nodes[z][y][x]
    for k in range(2):
        for j in range(2):
            for i in range(2):
                nodes[k, j, i] = (i, j, k)
    nodes[1, 1, 1] += (0.3, 0.2, 0.25)
    nodes[0, 1, 0] += (0.15, -0.1, 0.05)
    nodes[1, 0, 1] += (-0.1, 0.1, 0.2)
    f = O.Forest(3, p, N, (1, 1, 1), (0.0,) * 3, (1.0,) * 3, (1, 1, 1), 1)
    f.set_nodes(nodes)
    u = f.project_ic(O.IC_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1.0])
    rng = np.random.default_rng(50 + p)
    u[0, :, 1:, :] = 0.6 * rng.standard_normal(u[0, :, 1:, :].shape)
    before = u.copy()
    m0 = _physical_means3(u, nodes, p, N)
    assert m0[:, 0].min() > 0.2
    assert np.abs(m0 - before[0, :, 0, :].T).max() > 1e-3
    f.limit(u)
    np.testing.assert_allclose(_physical_means3(u, nodes, p, N), m0, rtol=1e-13, atol=1e-13)
    assert np.abs(u[0, :, 0, :] - before[0, :, 0, :]).max() > 1e-6
