"""Pins of the oracle's basis, quadrature, inheritance operators, fluxes and
time integrator against closed forms, numpy's independent Legendre routines
and brute force.  CPU only."""
import math
import os

import numpy as np
import pytest

import oracle as O
from tests import refmath as RM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gauss_legendre_closed_forms():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "gauss_legendre.txt")) if l.strip() and not l.startswith("#")]
    for q in (2, 3, 4, 5):
        ref = np.array([[float(r[1]), float(r[2])] for r in rows if int(r[0]) == q])
        x, w = O.gauss_legendre(q)
        np.testing.assert_allclose(x, ref[:, 0], rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, ref[:, 1], rtol=0, atol=4e-16)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_gauss_legendre_exactness_and_numpy(q):
    x, w = O.gauss_legendre(q)
    xn, wn = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, xn, atol=1e-15)
    np.testing.assert_allclose(w, wn, atol=1e-15)
    for k in range(2 * q):  # monomials up to degree 2q-1 integrate exactly
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


def test_legendre_values_against_numpy():
    for n in range(6):
        for xv in (-1.0, -0.7, -0.1, 0.0, 0.3, 0.9, 1.0):
            assert abs(O.legendre(n, xv) - RM.leg(n, xv)) < 1e-15
            assert abs(O.legendre_deriv(n, xv) - RM.dleg(n, xv)) < 1e-13
        assert O.legendre(n, 1.0) == 1.0
        assert O.legendre(n, -1.0) == (-1.0) ** n
    # closed forms P2 = (3x^2-1)/2, P3 = (5x^3-3x)/2
    assert abs(O.legendre(2, 0.4) - (3 * 0.16 - 1) / 2) < 1e-16
    assert abs(O.legendre(3, 0.4) - (5 * 0.064 - 1.2) / 2) < 1e-16


@pytest.mark.parametrize("dim,p", [(2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_mode_order(dim, p):
    e = O.mode_exponents(dim, p)
    assert len(e) == math.comb(p + dim, dim)
    assert [tuple(r) for r in e.tolist()] == RM.graded_modes(dim, p)
    if dim == 2 and p == 2:
        assert [tuple(r[:2]) for r in e.tolist()] == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_split_matrix_brute_force(dim, p):
    """Eq. 11-12: the child polynomial S^i K equals the parent polynomial on
    the child (the total-degree space is closed under the affine map)."""
    rng = np.random.default_rng(7 + dim * 10 + p)
    modes = RM.graded_modes(dim, p)
    for child in range(2 ** dim):
        S = O.split_matrix(dim, p, child)
        Kp = rng.standard_normal((1, len(modes)))
        Kc = (S @ Kp[0])[None, :]
        xi_c = rng.uniform(-1, 1, size=(20, dim))
        off = np.array([0.5 if (child >> a) & 1 else -0.5 for a in range(dim)])
        xi_p = off + 0.5 * xi_c
        np.testing.assert_allclose(RM.eval_cell(Kc, modes, xi_c), RM.eval_cell(Kp, modes, xi_p), atol=1e-13)


@pytest.mark.parametrize("dim,p", [(2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_combine_matrix_identities(dim, p):
    """Eq. 13-14: combine after split is the identity, combine keeps the
    mean, split-combine is a projection, and combine equals high-order
    quadrature of its definition."""
    nb = math.comb(p + dim, dim)
    modes = RM.graded_modes(dim, p)
    S = [O.split_matrix(dim, p, c) for c in range(2 ** dim)]
    C = [O.combine_matrix(dim, p, c) for c in range(2 ** dim)]
    np.testing.assert_allclose(sum(C[i] @ S[i] for i in range(2 ** dim)), np.eye(nb), atol=1e-14)
    rng = np.random.default_rng(3)
    kids = [rng.standard_normal(nb) for _ in range(2 ** dim)]
    parent = sum(C[i] @ kids[i] for i in range(2 ** dim))
    assert abs(parent[0] - np.mean([k[0] for k in kids])) < 1e-14
    P = np.block([[S[i] @ C[j] for j in range(2 ** dim)] for i in range(2 ** dim)])
    np.testing.assert_allclose(P @ P, P, atol=1e-13)
    # definition by brute-force quadrature over each child region
    for i in range(2 ** dim):
        off = np.array([0.5 if (i >> a) & 1 else -0.5 for a in range(dim)])
        pts, wts = RM.tensor_gauss(dim, 8)
        xp = off + 0.5 * pts
        ref = np.zeros((nb, nb))
        for l, ml in enumerate(modes):
            for j, mj in enumerate(modes):
                ref[l, j] = np.sum(wts * RM.phi(ml, xp) * RM.phi(mj, pts)) * 2.0 ** (-dim) / RM.ref_mass(ml, dim)
        np.testing.assert_allclose(C[i], ref, atol=1e-14)


def test_p0_split_combine_are_copy_and_average():
    for dim in (2, 3):
        for c in range(2 ** dim):
            assert O.split_matrix(dim, 0, c)[0, 0] == pytest.approx(1.0, abs=1e-15)
            assert O.combine_matrix(dim, 0, c)[0, 0] == pytest.approx(2.0 ** -dim, abs=1e-16)


def test_euler_flux_hand_values():
    # rho=2, rho u=1, rho v=-0.5, E=5 -> u=0.5, v=-0.25, p=0.4*(5-0.3125)=1.875
    u = [2.0, 1.0, -0.5, 5.0]
    fx = O.euler_flux(2, 1.4, u, 0)
    fy = O.euler_flux(2, 1.4, u, 1)
    np.testing.assert_allclose(fx, [1.0, 2.375, -0.25, 3.4375], atol=1e-15)
    np.testing.assert_allclose(fy, [-0.5, -0.25, 0.125 + 1.875, -0.25 * 6.875], atol=1e-15)
    # 3-D: rho=1, momenta (1,2,3), E=10 -> p = 0.4*(10-7) = 1.2
    u3 = [1.0, 1.0, 2.0, 3.0, 10.0]
    np.testing.assert_allclose(O.euler_flux(3, 1.4, u3, 2), [3.0, 3.0, 6.0, 9.0 + 1.2, 3.0 * 11.2], atol=1e-14)


def test_rusanov_consistency_antisymmetry_dissipation():
    rng = np.random.default_rng(11)
    for dim in (2, 3):
        for _ in range(20):
            rho = rng.uniform(0.5, 2)
            vel = rng.uniform(-1, 1, dim)
            p = rng.uniform(0.5, 2)
            u = np.concatenate([[rho], rho * vel, [p / 0.4 + 0.5 * rho * vel @ vel]])
            rho2 = rng.uniform(0.5, 2)
            vel2 = rng.uniform(-1, 1, dim)
            p2 = rng.uniform(0.5, 2)
            u2 = np.concatenate([[rho2], rho2 * vel2, [p2 / 0.4 + 0.5 * rho2 * vel2 @ vel2]])
            for axis in range(dim):
                for sign in (-1, 1):
                    # consistency: Fhat(U, U, n) = F(U) . n
                    np.testing.assert_allclose(O.rusanov(dim, 1.4, u, u, axis, sign),
                                               sign * O.euler_flux(dim, 1.4, u, axis), rtol=0, atol=1e-15)
                    a = O.rusanov(dim, 1.4, u, u2, axis, sign)
                    b = O.rusanov(dim, 1.4, u2, u, axis, -sign)
                    assert np.array_equal(a, -b)  # bitwise conservation
                    # dissipative sign: the jump term points from U- towards U+
                    central = 0.5 * sign * (O.euler_flux(dim, 1.4, u, axis) + O.euler_flux(dim, 1.4, u2, axis))
                    diss = a - central
                    assert np.dot(diss, u2 - u) <= 0.0


def test_rk3_amplification_polynomial():
    """Shu-Osher SSP-RK3 on y' = lambda y has amplification 1+z+z^2/2+z^3/6."""
    for z in (-0.3, -1.0, -2.5, 0.2, 1.1):
        lam, dt = z / 0.05, 0.05
        y = np.array([1.0, -2.0, 0.5])
        y1 = O.rk_combine(0, dt, y, y, lam * y)
        y2 = O.rk_combine(1, dt, y, y1, lam * y1)
        y3 = O.rk_combine(2, dt, y, y2, lam * y2)
        np.testing.assert_allclose(y3, (1 + z + z * z / 2 + z ** 3 / 6) * y, rtol=1e-14)
