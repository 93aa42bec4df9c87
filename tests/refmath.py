"""Independent reference mathematics for pinning the oracle.

Nothing here calls the oracle: Legendre values come from numpy's own
``numpy.polynomial.legendre`` routines and integrals from high-order
numpy Gauss rules, so that a mistake in the oracle's basis, quadrature or
projection code shows up as a disagreement.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def leg(n, x):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(x, c)


def dleg(n, x):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(x, npleg.legder(c))


def graded_modes(dim, p):
    """Total-degree exponent list in graded order: |m| ascending, then m_x
    descending, then m_y descending."""
    out = []
    for s in range(p + 1):
        for mx in range(s, -1, -1):
            if dim == 2:
                out.append((mx, s - mx, 0))
            else:
                for my in range(s - mx, -1, -1):
                    out.append((mx, my, s - mx - my))
    return out


def phi(m, xi):
    """phi_m at points xi (..., dim)."""
    xi = np.asarray(xi, dtype=float)
    v = np.ones(xi.shape[:-1])
    for a in range(xi.shape[-1]):
        v = v * leg(m[a], xi[..., a])
    return v


def eval_cell(coef, modes, xi):
    """coef (nv, nb) evaluated at xi (..., dim) -> (..., nv)."""
    basis = np.stack([phi(m, xi) for m in modes], axis=-1)  # (..., nb)
    return basis @ coef.T


def tensor_gauss(dim, q):
    x, w = npleg.leggauss(q)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    wg = np.meshgrid(*([w] * dim), indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=-1)
    wts = np.prod(np.stack([g.ravel() for g in wg], axis=-1), axis=-1)
    return pts, wts


def ref_mass(m, dim):
    return np.prod([2.0 / (2 * m[a] + 1) for a in range(dim)])


def project_box(func, dim, modes, cell_lo, cell_size, box_lo, box_hi, q=10):
    """(1/M_l) int_{box} phi_l(xi_cell(x)) func(x) dx / |J_cell| for a
    function of physical points; returns (nv, nb)."""
    pts, wts = tensor_gauss(dim, q)
    box_lo = np.asarray(box_lo, float)
    box_hi = np.asarray(box_hi, float)
    x = box_lo + 0.5 * (pts + 1.0) * (box_hi - box_lo)
    vol_box = np.prod(box_hi - box_lo)
    vol_cell = np.prod(np.asarray(cell_size, float) * np.ones(dim))
    xi = 2.0 * (x - np.asarray(cell_lo, float)) / np.asarray(cell_size, float) - 1.0
    vals = func(x)  # (npts, nv)
    out = np.zeros((vals.shape[1], len(modes)))
    for l, m in enumerate(modes):
        out[:, l] = (wts * phi(m, xi)) @ vals * (vol_box / 2 ** dim) / (vol_cell / 2 ** dim) / ref_mass(m, dim)
    return out


def euler_primitives(u, dim, gamma):
    rho = u[..., 0]
    vel = np.stack([u[..., 1 + a] / rho for a in range(dim)], axis=-1)
    p = (gamma - 1.0) * (u[..., dim + 1] - 0.5 * rho * np.sum(vel ** 2, axis=-1))
    return rho, vel, p
