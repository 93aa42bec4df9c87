"""Oracle: plain FP64 CPU implementation of the block-AMR explicit DG method.

THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU library never does,
and the two share no code.  The C sources next to this file follow the
paper's definitions one cell at a time (see ``oracle.h`` for the list of
passages); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = ["basis.c", "forest.c", "solver.c"]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_OUTFLOW, BC_DIRICHLET = 0, 1, 2
HANG_PAPER, HANG_CONSERVATIVE = 0, 1
IC_VORTEX, IC_SEDOV, IC_UNIFORM, IC_XWAVE, IC_COSINE, IC_EXP = 0, 1, 2, 3, 4, 5
EQ_EULER, EQ_ADVECTION, EQ_DIFFUSION = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", _LIB_PATH + ".tmp"] + [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        L.orc_legendre.restype = ctypes.c_double
        L.orc_legendre.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_legendre_deriv.restype = ctypes.c_double
        L.orc_legendre_deriv.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_num_modes.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_mode_exponents.argtypes = [ctypes.c_int, ctypes.c_int, ip]
        L.orc_split_matrix.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_combine_matrix.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_euler_flux.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp]
        L.orc_rusanov.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, ip,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_advection.argtypes = [vp, dp]
        L.orc_set_diffusion.argtypes = [vp, ctypes.c_double, dp]
        L.orc_set_time.argtypes = [vp, ctypes.c_double]
        L.orc_set_frames.argtypes = [vp, ip]
        L.orc_set_frames.restype = ctypes.c_int
        L.orc_set_nodes.argtypes = [vp, dp]
        L.orc_set_nodes.restype = ctypes.c_int
        L.orc_get_time.argtypes = [vp]
        L.orc_get_time.restype = ctypes.c_double
        L.orc_upwind.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.orc_upwind.restype = ctypes.c_double
        L.orc_num_leaves.argtypes = [vp]
        L.orc_leaf_keys.argtypes = [vp, ip]
        L.orc_state_len.restype = ctypes.c_long
        L.orc_state_len.argtypes = [vp]
        L.orc_guard_len.restype = ctypes.c_long
        L.orc_guard_len.argtypes = [vp]
        L.orc_plan_adapt.argtypes = [vp, ctypes.POINTER(ctypes.c_byte)]
        L.orc_apply_adapt.argtypes = [vp, dp, dp]
        L.orc_project_ic.argtypes = [vp, ctypes.c_int, dp, ctypes.c_double, dp]
        L.orc_fill_guards.argtypes = [vp, dp, dp]
        L.orc_residual.argtypes = [vp, dp, dp, dp]
        L.orc_rk_combine.argtypes = [ctypes.c_long, ctypes.c_int, ctypes.c_double, dp, dp, dp, dp]
        L.orc_max_rate.restype = ctypes.c_double
        L.orc_max_rate.argtypes = [vp, dp]
        L.orc_dt.restype = ctypes.c_double
        L.orc_dt.argtypes = [vp, dp, ctypes.c_double]
        L.orc_totals.argtypes = [vp, dp, dp]
        L.orc_limit_positivity.argtypes = [vp, dp]
        L.orc_indicator.argtypes = [vp, dp, dp]
        L.orc_step.restype = ctypes.c_double
        L.orc_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_errors.argtypes = [vp, dp, ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# ---------------------------------------------------------------- basis pieces
def legendre(n: int, x: float) -> float:
    return lib().orc_legendre(n, x)


def legendre_deriv(n: int, x: float) -> float:
    return lib().orc_legendre_deriv(n, x)


def gauss_legendre(q: int):
    x = np.zeros(q)
    w = np.zeros(q)
    lib().orc_gauss_legendre(q, _dp(x), _dp(w))
    return x, w


def mode_exponents(dim: int, p: int) -> np.ndarray:
    nb = lib().orc_num_modes(dim, p)
    e = np.zeros((nb, 3), dtype=np.int32)
    lib().orc_mode_exponents(dim, p, _ip(e))
    return e


def split_matrix(dim: int, p: int, child: int) -> np.ndarray:
    nb = lib().orc_num_modes(dim, p)
    S = np.zeros((nb, nb))
    lib().orc_split_matrix(dim, p, child, _dp(S))
    return S


def combine_matrix(dim: int, p: int, child: int) -> np.ndarray:
    nb = lib().orc_num_modes(dim, p)
    C = np.zeros((nb, nb))
    lib().orc_combine_matrix(dim, p, child, _dp(C))
    return C


def euler_flux(dim: int, gamma: float, u, axis: int) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(dim + 2)
    lib().orc_euler_flux(dim, gamma, _dp(u), axis, _dp(f))
    return f


def rusanov(dim: int, gamma: float, um, up, axis: int, sign: int) -> np.ndarray:
    um = np.ascontiguousarray(um, dtype=np.float64)
    up = np.ascontiguousarray(up, dtype=np.float64)
    f = np.zeros(dim + 2)
    lib().orc_rusanov(dim, gamma, _dp(um), _dp(up), axis, sign, _dp(f))
    return f


def upwind(vel, um: float, up: float, axis: int, sign: int) -> float:
    v = np.ascontiguousarray(list(vel) + [0.0] * (3 - len(vel)), dtype=np.float64)
    return lib().orc_upwind(_dp(v), um, up, axis, sign)


def rk_combine(stage: int, dt: float, un, us, r) -> np.ndarray:
    un, us, r = (np.ascontiguousarray(a, dtype=np.float64) for a in (un, us, r))
    out = np.zeros_like(un)
    lib().orc_rk_combine(un.size, stage, dt, _dp(un), _dp(us), _dp(r), _dp(out))
    return out


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int):
    lib().orc_set_threads(n)


# ---------------------------------------------------------------- forest
class Forest:
    """A forest of block trees with its DG state layout (see oracle.h)."""

    def __init__(self, dim, p, n_cell, roots, lo, hi, bc, max_level, gamma=1.4,
                 hanging=HANG_PAPER, equation=EQ_EULER, velocity=(1.0, 1.0, 1.0), nu=1.0,
                 avec=(-1.0, 1.0, 0.0)):
        roots = np.array(list(roots) + [1] * (3 - len(roots)), dtype=np.int32)
        lo = np.array(list(lo) + [0.0] * (3 - len(lo)), dtype=np.float64)
        hi = np.array(list(hi) + [1.0] * (3 - len(hi)), dtype=np.float64)
        bc = np.array(list(bc) + [0] * (3 - len(bc)), dtype=np.int32)
        self.dim, self.p, self.N = dim, p, n_cell
        self.gamma = gamma
        self.nv = dim + 2
        self.nb = lib().orc_num_modes(dim, p)
        self.ptr = lib().orc_create(dim, p, n_cell, _ip(roots), _dp(lo), _dp(hi), _ip(bc),
                                    max_level, gamma, hanging)
        if not self.ptr:
            raise ValueError("oracle: invalid forest description")
        self.equation = equation
        if equation == EQ_ADVECTION:
            self.velocity = np.array(list(velocity) + [0.0] * (3 - len(velocity)), dtype=np.float64)
            lib().orc_set_advection(self.ptr, _dp(self.velocity))
            self.nv = 1
        elif equation == EQ_DIFFUSION:
            self.nu = nu
            self.avec = np.array(list(avec) + [0.0] * (3 - len(avec)), dtype=np.float64)[:3]
            lib().orc_set_diffusion(self.ptr, nu, _dp(self.avec))
            self.nv = 1

    def set_frames(self, codes):
        """Rotation code of each root's local frame (see oracle.h)."""
        c = np.ascontiguousarray(codes, dtype=np.int32)
        if lib().orc_set_frames(self.ptr, _ip(c)) != 0:
            raise ValueError("oracle: frames refused")

    def set_nodes(self, xy):
        """Bilinear (3-D: trilinear) root blocks (Sec. 3.3, Eq. 6) from the
        root grid nodes, shape (roots_y + 1, roots_x + 1, 2) or (roots_z + 1,
        roots_y + 1, roots_x + 1, 3) (see oracle.h)."""
        a = np.ascontiguousarray(xy, dtype=np.float64)
        if lib().orc_set_nodes(self.ptr, _dp(a)) != 0:
            raise ValueError("oracle: nodes refused")

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_destroy(self.ptr)
            self.ptr = None

    @property
    def n_leaves(self) -> int:
        return lib().orc_num_leaves(self.ptr)

    @property
    def time(self) -> float:
        return lib().orc_get_time(self.ptr)

    @time.setter
    def time(self, t: float):
        lib().orc_set_time(self.ptr, t)

    @property
    def ncell(self) -> int:
        return self.N ** self.dim

    def keys(self) -> np.ndarray:
        k = np.zeros((self.n_leaves, 5), dtype=np.int32)
        lib().orc_leaf_keys(self.ptr, _ip(k))
        return k

    def state_shape(self):
        return (self.n_leaves, self.nv, self.nb, self.ncell)

    def guard_shape(self):
        return (self.n_leaves, 2 * self.dim, self.nv, self.nb, self.N ** (self.dim - 1))

    def zeros(self):
        return np.zeros(self.state_shape())

    def adapt(self, flags, u_old=None):
        flags = np.ascontiguousarray(flags, dtype=np.int8)
        assert flags.size == self.n_leaves
        n_new = lib().orc_plan_adapt(self.ptr, flags.ctypes.data_as(ctypes.POINTER(ctypes.c_byte)))
        if u_old is None:
            u_old = self.zeros()
        u_old = np.ascontiguousarray(u_old, dtype=np.float64)
        u_new = np.zeros((n_new, self.nv, self.nb, self.ncell))
        lib().orc_apply_adapt(self.ptr, _dp(u_old), _dp(u_new))
        return u_new

    def project_ic(self, kind, params, t=0.0):
        u = self.zeros()
        prm = np.zeros(8)
        prm[: len(params)] = params
        lib().orc_project_ic(self.ptr, kind, _dp(prm), t, _dp(u))
        return u

    def fill_guards(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        g = np.zeros(self.guard_shape())
        lib().orc_fill_guards(self.ptr, _dp(u), _dp(g))
        return g

    def residual(self, u, g=None):
        u = np.ascontiguousarray(u, dtype=np.float64)
        if g is None:
            g = self.fill_guards(u)
        r = np.zeros_like(u)
        lib().orc_residual(self.ptr, _dp(u), _dp(np.ascontiguousarray(g)), _dp(r))
        return r

    def max_rate(self, u) -> float:
        return lib().orc_max_rate(self.ptr, _dp(np.ascontiguousarray(u, dtype=np.float64)))

    def dt(self, u, cfl) -> float:
        return lib().orc_dt(self.ptr, _dp(np.ascontiguousarray(u, dtype=np.float64)), cfl)

    def totals(self, u):
        t = np.zeros(self.nv)
        lib().orc_totals(self.ptr, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(t))
        return t

    def limit(self, u):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        lib().orc_limit_positivity(self.ptr, _dp(u))
        return u

    def indicator(self, u):
        eta = np.zeros(self.n_leaves)
        lib().orc_indicator(self.ptr, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(eta))
        return eta

    def step(self, u, cfl=0.1, dt=0.0, limiter=False) -> float:
        """One SSP-RK3 step in place; returns the dt used."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        return lib().orc_step(self.ptr, cfl, dt, 1 if limiter else 0, _dp(u))

    def errors(self, u, kind, params, t):
        prm = np.zeros(8)
        prm[: len(params)] = params
        l1 = np.zeros(self.nv)
        l2 = np.zeros(self.nv)
        lib().orc_errors(self.ptr, _dp(np.ascontiguousarray(u, dtype=np.float64)), kind, _dp(prm), t,
                         _dp(l1), _dp(l2))
        return l1, l2
