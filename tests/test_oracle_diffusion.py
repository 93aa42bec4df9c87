"""Pins of the oracle's diffusion operator (Sec. 5.2: u_t = nu div grad u,
symmetric interior-penalty DG, Dirichlet data from the exact solution
exp(a . x + nu |a|^2 t)): exactness on polynomials, symmetry and sign of
the operator, the exact solution's observed order, and the time step.
Expected values are closed forms or properties; nothing here re-derives
the operator.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from tests import refmath as RM


def _forest(p, N, roots=(2, 2), bc=(2, 2), refine=(), nu=1.0, avec=(-1.0, 1.0), lo=(0.0, 0.0), hi=(1.0, 1.0),
            levels=2, dim=2):
    f = O.Forest(dim, p, N, roots, lo, hi, bc, levels, equation=O.EQ_DIFFUSION, nu=nu, avec=avec)
    if refine:
        fl = np.zeros(f.n_leaves, np.int8)
        fl[list(refine)] = 1
        f.adapt(fl)
    return f


def _project_poly(f, func, roots, lo, hi):
    """Cell coefficients of a polynomial of degree <= p (exact L2
    projection by high-order numpy Gauss quadrature, from the keys)."""
    d, N, p = f.dim, f.N, f.p
    modes = RM.graded_modes(d, p)
    u = f.zeros()
    keys = f.keys()
    R = list(roots) + [1] * (3 - d)
    for li, (tree, level, i, j, k) in enumerate(keys):
        r = [tree % R[0], (tree // R[0]) % R[1], tree // (R[0] * R[1])]
        edge = np.array([(hi[a] - lo[a]) / R[a] / 2 ** (level - 1) for a in range(d)])
        corner = np.array([lo[a] + r[a] * (hi[a] - lo[a]) / R[a] + (i, j, k)[a] * edge[a] for a in range(d)])
        h = edge / N
        for c in range(N ** d):
            ijk = np.array([c % N, (c // N) % N, c // (N * N)][:d])
            clo = corner + ijk * h
            coef = RM.project_box(lambda x: func(x)[:, None], d, modes, clo, h, clo, clo + h, q=p + 2)
            u[li, 0, :, c] = coef[0]
    return u


@pytest.mark.parametrize("p", [1, 2, 3])
def test_harmonic_polynomials_have_zero_residual(p):
    """u = 1 with a = 0 (so the Dirichlet data is 1) on a forest with
    hanging faces: the gradient, the jumps and the boundary mismatch are
    zero, so every term of the operator vanishes."""
    f = _forest(p, 4, refine=[0], avec=(0.0, 0.0))
    u = f.project_ic(O.IC_EXP, [])
    np.testing.assert_allclose(u[:, 0, 0, :], 1.0, atol=1e-15)
    r = f.residual(u)
    assert np.abs(r).max() < 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
def test_periodic_polynomial_consistency(p):
    """Consistency across interior and hanging faces: a linear u on a
    periodic forest with root 0 refined.  Away from the periodic seam (where
    a linear function jumps) every neighbour polynomial and guard cell
    (copy, split, combine of a linear function) is the same linear
    function, so the operator returns the projection of div grad u = 0."""
    roots, lo, hi = (2, 2), (0.0, 0.0), (1.0, 1.0)
    f = _forest(p, 4, roots=roots, bc=(0, 0), refine=[0])
    u = _project_poly(f, lambda x: 0.3 + 0.7 * x[:, 0] - 0.2 * x[:, 1], roots, lo, hi)
    r = f.residual(u)
    # a linear function is not periodic: only cells away from the periodic
    # seam x = 0 / 1, y = 0 / 1 see a smooth neighbourhood
    keys = f.keys()
    N = f.N
    interior = []
    for li, (tree, level, i, j, k) in enumerate(keys):
        R = roots[0]
        rx, ry = tree % R, tree // R
        n = 2 ** (level - 1) * N
        for c in range(N * N):
            gx = (rx * 2 ** (level - 1) + i) * N + c % N
            gy = (ry * 2 ** (level - 1) + j) * N + c // N
            tot = R * n
            if 0 < gx < tot - 1 and 0 < gy < tot - 1:
                interior.append((li, c))
    assert len(interior) > 0
    vals = np.array([np.abs(r[li, 0, :, c]).max() for li, c in interior])
    assert vals.max() < 1e-9


@pytest.mark.parametrize("p", [2, 3])
def test_quadratic_gives_the_projection_of_its_laplacian(p):
    """u = x^2 + 2 y^2 (Laplacian 6) with nu = 1.5 on a periodic forest
    with root 0 refined, at the cells away from the periodic seam: the SIPG
    operator is consistent, so R is the projection of nu * 6: mode 0 = 9,
    every other mode 0, also across the hanging faces."""
    roots, lo, hi = (2, 2), (0.0, 0.0), (1.0, 1.0)
    f = _forest(p, 4, roots=roots, bc=(0, 0), refine=[0], nu=1.5)
    u = _project_poly(f, lambda x: x[:, 0] ** 2 + 2 * x[:, 1] ** 2, roots, lo, hi)
    r = f.residual(u)
    keys = f.keys()
    N = f.N
    checked = 0
    for li, (tree, level, i, j, k) in enumerate(keys):
        rx, ry = tree % 2, tree // 2
        for c in range(N * N):
            gx = (rx * 2 ** (level - 1) + i) * N + c % N
            gy = (ry * 2 ** (level - 1) + j) * N + c // N
            tot = 2 * 2 ** (level - 1) * N
            if 0 < gx < tot - 1 and 0 < gy < tot - 1:
                assert r[li, 0, 0, c] == pytest.approx(9.0, abs=1e-8)
                assert np.abs(r[li, 0, 1:, c]).max() < 1e-8
                checked += 1
    assert checked > 50


@pytest.mark.parametrize("p", [1, 2, 3])
def test_operator_is_symmetric_and_negative_semidefinite(p):
    """On a periodic conforming forest the map u -> R(u) is linear, and
    M R is symmetric (SIPG is the symmetric form) and negative
    semi-definite with the constants as its kernel."""
    f = _forest(p, 2, roots=(2, 2), bc=(0, 0), avec=(0.0, 0.0), levels=1)
    shape = f.state_shape()
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = f.residual(e.reshape(shape)).ravel()
    modes = RM.graded_modes(2, p)
    Mm = np.array([RM.ref_mass(m, 2) for m in modes])
    Md = np.broadcast_to(Mm[None, None, :, None], shape).ravel()
    MA = Md[:, None] * A
    assert np.abs(MA - MA.T).max() <= 1e-12 * np.abs(MA).max()
    ev = np.linalg.eigvalsh(0.5 * (MA + MA.T))
    assert ev.max() <= 1e-10 * np.abs(ev).max()
    assert np.sum(np.abs(ev) <= 1e-10 * np.abs(ev).max()) == 1  # only the constant


@pytest.mark.parametrize("p", [1, 2, 3])
def test_exact_solution_order(p):
    """Sec. 5.2's exact solution exp(-x + y + 2t) on the unit square with
    Dirichlet data: observed L2 order p + 1 (dt ~ h^2, well inside the
    explicit stability bound, so the time error is negligible)."""
    errs = []
    c = {1: 0.01, 2: 0.003, 3: 0.0012}[p]
    for N in (4, 8):
        f = _forest(p, N, roots=(1, 1), levels=1)
        u = f.project_ic(O.IC_EXP, [])
        T = 0.01
        n = int(math.ceil(T / (c / N ** 2)))
        for _ in range(n):
            f.step(u, dt=T / n)
        assert f.time == pytest.approx(T, rel=1e-12)
        errs.append(f.errors(u, O.IC_EXP, [], T)[1][0])
    assert math.log2(errs[0] / errs[1]) >= p + 1 - 0.2, errs


def test_exact_solution_on_a_two_level_forest():
    """The same exact solution across hanging faces (root 0 refined): the
    error stays at the level of the uniform coarse forest, and the state
    follows exp(2t) growth (the mean over the square grows by e^{2t})."""
    p, N, T = 2, 4, 0.01
    f = _forest(p, N, refine=[0])
    u = f.project_ic(O.IC_EXP, [])
    n = int(math.ceil(T / (0.003 / (2 * N) ** 2 / 4)))
    for _ in range(n):
        f.step(u, dt=T / n)
    l2 = f.errors(u, O.IC_EXP, [], T)[1][0]
    g = _forest(p, N)
    v = g.project_ic(O.IC_EXP, [])
    for _ in range(n):
        g.step(v, dt=T / n)
    l2c = g.errors(v, O.IC_EXP, [], T)[1][0]
    assert l2 < 2.0 * l2c
    mean = f.totals(u)[0]
    exact = (1 - math.exp(-1)) * (math.e - 1) * math.exp(2 * T)  # int exp(-x) dx * int exp(y) dy * e^{2T}
    assert mean == pytest.approx(exact, rel=1e-4)


def test_diffusive_time_step_closed_form():
    """dt = cfl / (nu sum_a 1/h_a^2) at the finest cells."""
    f = _forest(2, 4, refine=[0], nu=0.5)
    u = f.project_ic(O.IC_EXP, [])
    h = 1.0 / 16  # root 0 refined: 2 x 2 leaves of 4 cells on a 0.5 root
    assert f.dt(u, 0.01) == pytest.approx(0.01 / (0.5 * 2 / h ** 2), rel=1e-14)
