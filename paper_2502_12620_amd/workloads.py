"""Seeded, synthetic workload descriptions shared by the GPU path, the tests
and the benchmark.

This module holds no arithmetic of the DG method: only forest shapes,
initial-refinement rules (by root/leaf geometry), analytic initial-condition
parameters, step counts and the random draws of the batched and served
workloads.  Every workload is synthetic; there is no dataset.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, OUTFLOW, DIRICHLET = 0, 1, 2
IC_VORTEX, IC_SEDOV, IC_UNIFORM, IC_XWAVE, IC_COSINE, IC_EXP = 0, 1, 2, 3, 4, 5
EQ_EULER, EQ_ADVECTION, EQ_DIFFUSION = 0, 1, 2


@dataclass
class Workload:
    name: str
    dim: int
    degree: int
    n_cell: int
    roots: tuple
    lo: tuple
    hi: tuple
    bc: tuple
    max_level: int
    ic_kind: int
    ic_params: list
    steps: int
    cfl: float = 0.1
    gamma: float = 1.4
    limiter: bool = False
    regrid_every: int = 0
    refine_above: float = 1.2
    coarsen_below: float = 1.01
    # list of refinement passes; each pass maps leaf keys -> flags
    initial_refinement: list = field(default_factory=list)
    equation: int = EQ_EULER
    velocity: tuple = (1.0, 1.0, 1.0)
    t_end: float = 0.0
    min_level: int = 1
    nu: float = 1.0
    exact_a: tuple = (-1.0, 1.0, 0.0)

    def desc(self) -> dict:
        return dict(dim=self.dim, degree=self.degree, n_cell=self.n_cell, roots=self.roots, lo=self.lo,
                    hi=self.hi, bc=self.bc, max_level=self.max_level, gamma=self.gamma)

    def leaf_boxes(self, keys):
        """Physical (lower corner, edge) of each leaf key (tree, level, i, j, k)."""
        d = self.dim
        roots = list(self.roots) + [1] * (3 - d)
        out = []
        for tree, level, i, j, k in np.asarray(keys):
            r = [tree % roots[0], (tree // roots[0]) % roots[1], tree // (roots[0] * roots[1])]
            idx = [i, j, k]
            root_edge = [(self.hi[a] - self.lo[a]) / roots[a] for a in range(d)]
            edge = np.array([root_edge[a] / 2 ** (level - 1) for a in range(d)])
            lo = np.array([self.lo[a] + r[a] * root_edge[a] + idx[a] * edge[a] for a in range(d)])
            out.append((lo, edge, int(level)))
        return out

    def dofs(self, n_leaves) -> int:
        nb = math.comb(self.degree + self.dim, self.dim)
        nv = 1 if self.equation in (EQ_ADVECTION, EQ_DIFFUSION) else self.dim + 2
        return n_leaves * nv * nb * self.n_cell ** self.dim


def refine_roots_near(centre, radius):
    """Flags +1 for the leaves whose centre lies within `radius` of `centre`."""
    def rule(w: Workload, keys):
        fl = []
        for lo, edge, _ in w.leaf_boxes(keys):
            c = lo + 0.5 * edge
            fl.append(1 if np.hypot(*(c - np.asarray(centre))) <= radius else 0)
        return np.array(fl, dtype=np.int8)
    return rule


def refine_all(w: Workload, keys):
    """Flags +1 for every leaf."""
    return np.ones(len(keys), dtype=np.int8)


def refine_touching(point, level=None):
    """Flags +1 for the leaves (optionally of one level) whose closed box
    contains `point`."""
    def rule(w: Workload, keys):
        fl = []
        for lo, edge, lv in w.leaf_boxes(keys):
            inside = all(lo[a] <= point[a] <= lo[a] + edge[a] for a in range(w.dim))
            fl.append(1 if inside and (level is None or lv == level) else 0)
        return np.array(fl, dtype=np.int8)
    return rule


# ---------------------------------------------------------------- the fixed workloads
def vortex_c1() -> Workload:
    """2-D isentropic vortex (strength 5, periodic [0,10]^2), single level:
    4x4 roots of 8x8 cells, P1, CFL 0.1, 20 steps."""
    return Workload("c1_vortex2d_p1_single_level", 2, 1, 8, (4, 4), (0.0, 0.0), (10.0, 10.0),
                    (PERIODIC, PERIODIC), 1, IC_VORTEX, [5.0, 5.0, 5.0, 1.0, 1.0, 10.0, 10.0], 20)


def vortex_c2() -> Workload:
    """2-D vortex, 2-level static AMR: 8x8 roots of 16x16 cells, roots with
    centre within 2.5 of (5,5) refined once (100 leaves), P2, 200 steps."""
    return Workload("c2_vortex2d_p2_two_level", 2, 2, 16, (8, 8), (0.0, 0.0), (10.0, 10.0),
                    (PERIODIC, PERIODIC), 2, IC_VORTEX, [5.0, 5.0, 5.0, 1.0, 1.0, 10.0, 10.0], 200,
                    initial_refinement=[refine_roots_near((5.0, 5.0), 2.5)])


def sedov_c3() -> Workload:
    """3-D Sedov-style blast on [0,1]^3: 4^3 roots of 8^3 cells, levels 1..3
    (176 leaves initially), rho = 1, p = 1e-5 except 1e3 in the 8 finest
    cells at the centre, outflow, P2, positivity limiter, regrid every 10
    steps, 100 steps."""
    c = (0.5, 0.5, 0.5)
    return Workload("c3_sedov3d_p2_amr", 3, 2, 8, (4, 4, 4), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    (OUTFLOW, OUTFLOW, OUTFLOW), 3, IC_SEDOV, [1e-5, 1e3, 0.5, 0.5, 0.5], 100,
                    limiter=True, regrid_every=10,
                    initial_refinement=[refine_touching(c), refine_touching(c, level=2)])


def convection_2d(degree: int = 2, n_cell: int = 8) -> Workload:
    """Linear scalar convection (Sec. 5.1, first root set): one square root
    block on the periodic [0,1]^2, velocity (1,1), u0 = [cos(2 pi x) - 1]
    [cos(2 pi y) - 1], refinement levels 3..5 driven by the block's largest
    cell average (refine above 3.0, coarsen below 1.0) every 10 steps,
    SSP-RK3 at CFL 0.1 to t = 1.  Degree and block size are not given in
    the paper; degree 2 with 8x8-cell blocks here."""
    w = Workload("f1_convection2d", 2, degree, n_cell, (1, 1), (0.0, 0.0), (1.0, 1.0), (PERIODIC, PERIODIC), 5,
                 IC_COSINE, [1.0, 1.0, 1.0, 1.0], 0, regrid_every=10, refine_above=3.0, coarsen_below=1.0,
                 initial_refinement=[refine_all, refine_all])
    w.equation, w.velocity, w.t_end, w.min_level = EQ_ADVECTION, (1.0, 1.0, 0.0), 1.0, 3
    return w


def convection_3d(degree: int = 1, n_cell: int = 4) -> Workload:
    """Linear scalar convection in 3-D (Sec. 5.1): one root block on the
    periodic [0,1]^3 refined to level 4, u0 = prod [cos(4 pi x_a) - 1],
    velocity (1,1,1), to t = 0.25."""
    w = Workload("f1_convection3d", 3, degree, n_cell, (1, 1, 1), (0.0,) * 3, (1.0,) * 3, (PERIODIC,) * 3, 4,
                 IC_COSINE, [2.0, 1.0, 1.0, 1.0], 0, initial_refinement=[refine_all, refine_all, refine_all])
    w.equation, w.velocity, w.t_end, w.min_level = EQ_ADVECTION, (1.0, 1.0, 1.0), 0.25, 4
    return w


def convection_2d_distorted(degree: int = 2, n_cell: int = 8) -> Workload:
    """The convection case of Sec. 5.1 on its second root set, four
    distorted root blocks.  The paper shows that set only as a figure: here
    a 2x2 root grid on the periodic unit square whose centre node is moved
    from (0.5, 0.5) to (0.6, 0.42), the boundary nodes staying on the box,
    so every root is a convex quadrilateral and the grid stays periodic.
    Everything else as convection_2d."""
    w = convection_2d(degree, n_cell)
    w.name = "f1_convection2d_distorted"
    w.roots = (2, 2)
    nodes = np.zeros((3, 3, 2))
    nodes[..., 0] = np.array([0.0, 0.5, 1.0])[None, :]
    nodes[..., 1] = np.array([0.0, 0.5, 1.0])[:, None]
    nodes[1, 1] = (0.6, 0.42)
    w.nodes = nodes
    w.initial_refinement = [refine_all]
    w.min_level = 2
    w.max_level = 4
    return w


def convection_2d_rotated(degree: int = 2, n_cell: int = 8) -> Workload:
    """The convection case of Sec. 5.1 on roots whose local frames are
    rotated against each other (the paper's third root set, an unstructured
    mesh shown only as a figure, has rotated roots): a 2x2 grid of square
    roots on the periodic unit square, each turned by a different number of
    quarter turns (frames 0, 1, 2, 3), levels 2..4 (the cell sizes of the
    first set).  Everything else as convection_2d."""
    w = convection_2d_distorted(degree, n_cell)
    w.name = "f1_convection2d_rotated"
    w.frames = [0, 1, 2, 3]
    del w.nodes
    return w


def diffusion_2d(degree: int = 2, n_cell: int = 6) -> Workload:
    """Diffusion (Sec. 5.2): u_t = div grad u on the unit square, one root
    block, Dirichlet data and initial state from exp(-x + y + 2t), 6x6-cell
    blocks, refinement levels 2..4 driven by the block's largest cell
    average (refine above 3.0, coarsen below 1.0) every 10 steps, SSP-RK3 at
    the diffusive CFL number 0.006 (dt = 0.006 h^2 / 2) to t = 0.2.  The
    degree is not given in the paper; 2 here."""
    w = Workload("f4_diffusion2d", 2, degree, n_cell, (1, 1), (0.0, 0.0), (1.0, 1.0), (DIRICHLET, DIRICHLET), 4,
                 IC_EXP, [], 0, cfl=0.006, regrid_every=10, refine_above=3.0, coarsen_below=1.0,
                 initial_refinement=[refine_all])
    w.equation, w.t_end, w.min_level = EQ_DIFFUSION, 0.2, 2
    w.nu, w.exact_a = 1.0, (-1.0, 1.0)
    return w


def regrid_flags(w: Workload, keys, eta):
    """Refinement flags of the convection and diffusion workloads from the block
    indicator: +1 above refine_above, -1 below coarsen_below, never below
    the minimum level."""
    flags = np.where(eta > w.refine_above, 1, np.where(eta < w.coarsen_below, -1, 0)).astype(np.int8)
    levels = np.asarray(keys)[:, 1]
    flags[(flags < 0) & (levels <= w.min_level)] = 0
    return flags


def roofline_2d(k: int, degree: int) -> Workload:
    """Uniform 2-D vortex forest of k x k roots of 16x16 cells (roofline sweep)."""
    L = 2.5 * k
    return Workload(f"rs_vortex2d_k{k}_p{degree}", 2, degree, 16, (k, k), (0.0, 0.0), (L, L),
                    (PERIODIC, PERIODIC), 1, IC_VORTEX, [5.0, L / 2, L / 2, 1.0, 1.0, L, L], 10)


def roofline_3d(k: int, degree: int) -> Workload:
    """Uniform 3-D extruded-vortex forest of k^3 roots of 8^3 cells."""
    L = 1.25 * k
    return Workload(f"rs_vortex3d_k{k}_p{degree}", 3, degree, 8, (k, k, k), (0.0, 0.0, 0.0), (L, L, L),
                    (PERIODIC, PERIODIC, PERIODIC), 1, IC_VORTEX, [5.0, L / 2, L / 2, 1.0, 1.0, L, L], 10)


def smooth_root_nodes(w: Workload, amp: float = 0.1):
    """Root grid nodes of w's uniform root grid moved by a smooth periodic
    displacement of amp root widths (each coordinate by amp h sin(2 pi x_b /
    L_b) over the other axes b), so that every root becomes a bilinear
    (trilinear) block and a periodic axis stays periodic.  Shape (ry + 1,
    rx + 1, 2) or (rz + 1, ry + 1, rx + 1, 3)."""
    d = w.dim
    r = list(w.roots[:d])
    axes = [np.linspace(w.lo[a], w.hi[a], r[a] + 1) for a in range(d)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]  # x varies fastest (last index)
    L = [w.hi[a] - w.lo[a] for a in range(d)]
    nodes = np.stack(grids, axis=-1)
    for a in range(d):
        h = L[a] / r[a]
        disp = np.ones_like(grids[0])
        for b in range(d):
            if b != a:
                disp = disp * np.sin(2.0 * np.pi * (grids[b] - w.lo[b]) / L[b])
        nodes[..., a] += amp * h * disp
    return nodes


def random_root_frames(w: Workload, seed: int = 31):
    """A seeded rotation code per root (4 frames in 2-D, 24 in 3-D)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(w.roots[:w.dim]))
    return [int(x) for x in rng.integers(0, 4 if w.dim == 2 else 24, n)]


def batched_forests(n: int = 512, seed: int = 2502):
    """The batched workload: n independent 2-D vortex forests.  Root count
    R ~ U{4..256} as nx x ny (nx the largest divisor of R not above sqrt R),
    root edge 2.5, 16x16 cells, degree ~ U{1,2,3}, strength ~ U[1,5],
    centre ~ U(domain), 20 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        R = int(rng.integers(4, 257))
        nx = max(d for d in range(1, int(math.isqrt(R)) + 1) if R % d == 0)
        ny = R // nx
        p = int(rng.integers(1, 4))
        eps = float(rng.uniform(1.0, 5.0))
        Lx, Ly = 2.5 * nx, 2.5 * ny
        cx, cy = float(rng.uniform(0, Lx)), float(rng.uniform(0, Ly))
        out.append(Workload(f"batch{i}", 2, p, 16, (nx, ny), (0.0, 0.0), (Lx, Ly), (PERIODIC, PERIODIC), 1,
                            IC_VORTEX, [eps, cx, cy, 1.0, 1.0, Lx, Ly], 20))
    return out


def served_requests(n: int = 1000, seed: int = 12620, rate: float = 200.0):
    """The served workload: a Poisson stream (mean `rate` requests/s) of
    2-D/3-D vortex solves.  Blocks ~ log-uniform in [16, 2048] (2-D 16x16
    cells, 3-D 8^3), degree ~ U{1,2,3}, steps ~ U{50..500}.  Returns
    (arrival_time_s, Workload) pairs."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        dim = int(rng.integers(2, 4))
        blocks = int(round(math.exp(rng.uniform(math.log(16), math.log(2048)))))
        p = int(rng.integers(1, 4))
        steps = int(rng.integers(50, 501))
        if dim == 2:
            nx = max(d for d in range(1, int(math.isqrt(blocks)) + 1) if blocks % d == 0)
            roots = (nx, blocks // nx)
            Lx, Ly = 2.5 * roots[0], 2.5 * roots[1]
            w = Workload(f"req{i}", 2, p, 16, roots, (0.0, 0.0), (Lx, Ly), (PERIODIC, PERIODIC), 1, IC_VORTEX,
                         [3.0, Lx / 2, Ly / 2, 1.0, 1.0, Lx, Ly], steps)
        else:
            c = round(blocks ** (1.0 / 3.0))
            c = max(2, c)
            roots = (c, c, max(1, blocks // (c * c)))
            L = [1.25 * r for r in roots]
            w = Workload(f"req{i}", 3, p, 8, roots, (0.0, 0.0, 0.0), tuple(L), (PERIODIC,) * 3, 1, IC_VORTEX,
                         [3.0, L[0] / 2, L[1] / 2, 1.0, 1.0, L[0], L[1]], steps)
        out.append((t, w))
    return out
