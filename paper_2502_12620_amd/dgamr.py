"""Thin Python binding of the dgamr C-ABI (``include/dgamr.h``).

Argument marshalling only: every step of the DG path runs in the HIP
library ``libdgamr.so``.  PyTorch supplies device memory and the current
HIP stream.  There is no fallback: if the library is missing, importing the
binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgamr.so")

OK, EINVAL, EUNSUPPORTED, EBALANCE, EHIP, ENONPHYSICAL, ESTATE, EFULL = 0, -1, -2, -3, -4, -5, -6, -7
BC_PERIODIC, BC_OUTFLOW, BC_DIRICHLET = 0, 1, 2
FP64, FP32 = 0, 1
HANG_PAPER, HANG_CONSERVATIVE = 0, 1
LIMITER_NONE, LIMITER_POSITIVITY = 0, 1
IC_VORTEX, IC_SEDOV, IC_UNIFORM, IC_XWAVE, IC_COSINE, IC_EXP = 0, 1, 2, 3, 4, 5
EQ_EULER, EQ_ADVECTION, EQ_DIFFUSION = 0, 1, 2
TUNE_STAGE_VARIANT, TUNE_VAR_SPLIT_MAX_CELLS, TUNE_SLAB_ROWS, TUNE_MFMA = 0, 1, 2, 3

EXPORTS = [
    "dgamr_create_forest", "dgamr_destroy_forest", "dgamr_num_leaves", "dgamr_leaf_keys",
    "dgamr_state_bytes", "dgamr_set_refinement", "dgamr_apply_refinement",
    "dgamr_fill_guardcells", "dgamr_dg_residual", "dgamr_rk_stage", "dgamr_compute_dt",
    "dgamr_step", "dgamr_run", "dgamr_conserved_totals", "dgamr_limit_positivity", "dgamr_indicator",
    "dgamr_project_ic", "dgamr_check_state", "dgamr_set_tuning", "dgamr_profile_enable", "dgamr_profile_read",
    "dgamr_pool_create", "dgamr_pool_destroy", "dgamr_pool_bytes", "dgamr_pool_admit", "dgamr_pool_release",
    "dgamr_pool_step", "dgamr_pool_dt", "dgamr_pool_stats", "dgamr_pool_set_shape", "dgamr_pool_set_lanes", "dgamr_pool_autotune",
    "dgamr_pools_capture", "dgamr_graph_launch", "dgamr_graph_destroy", "dgamr_run_capture",
    "dgamr_step_static", "dgamr_set_time", "dgamr_get_time", "dgamr_set_root_frames", "dgamr_set_root_nodes", "dgamr_math_probe",
    "dgamr_last_error",
]


class DgamrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dgamr error {code}: {msg}")
        self.code = code


class ForestDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("degree", ctypes.c_int), ("n_cell", ctypes.c_int),
        ("roots", ctypes.c_int * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3), ("max_level", ctypes.c_int), ("gamma", ctypes.c_double),
        ("precision", ctypes.c_int), ("hanging", ctypes.c_int), ("limiter", ctypes.c_int),
        ("equation", ctypes.c_int), ("velocity", ctypes.c_double * 3),
        ("diffusivity", ctypes.c_double), ("exact_a", ctypes.c_double * 3),
    ]


_lib = None


def lib():
    """Load libdgamr.so (built by paper_2502_12620_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2502_12620_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64p, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)
        L.dgamr_create_forest.argtypes = [ctypes.POINTER(ForestDesc), ctypes.POINTER(vp)]
        L.dgamr_destroy_forest.argtypes = [vp]
        L.dgamr_num_leaves.argtypes = [vp, i64p]
        L.dgamr_leaf_keys.argtypes = [vp, vp]
        L.dgamr_state_bytes.argtypes = [vp, sz, sz, sz, sz]
        L.dgamr_set_refinement.argtypes = [vp, vp, i64p]
        L.dgamr_apply_refinement.argtypes = [vp, vp, vp, vp]
        L.dgamr_fill_guardcells.argtypes = [vp, vp, vp, vp]
        L.dgamr_dg_residual.argtypes = [vp, vp, vp, vp, vp]
        L.dgamr_rk_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.dgamr_compute_dt.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp]
        L.dgamr_step.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp]
        L.dgamr_step_static.argtypes = [vp, ctypes.c_double, vp, vp, vp]
        L.dgamr_set_time.argtypes = [vp, ctypes.c_double]
        L.dgamr_set_root_frames.argtypes = [vp, vp]
        L.dgamr_set_root_nodes.argtypes = [vp, vp]
        L.dgamr_math_probe.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int64, vp]
        L.dgamr_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.dgamr_run.argtypes = [vp, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp]
        L.dgamr_conserved_totals.argtypes = [vp, vp, vp, vp, vp]
        L.dgamr_limit_positivity.argtypes = [vp, vp, vp]
        L.dgamr_indicator.argtypes = [vp, vp, vp, vp, vp]
        L.dgamr_project_ic.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp, vp]
        L.dgamr_check_state.argtypes = [vp, vp, i64p, vp, vp]
        L.dgamr_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_long]
        L.dgamr_profile_enable.argtypes = [vp, ctypes.c_int]
        L.dgamr_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64p]
        i32, i32p = ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)
        L.dgamr_pool_create.argtypes = [ctypes.POINTER(ForestDesc), ctypes.c_int64, i32, ctypes.POINTER(vp)]
        L.dgamr_pool_destroy.argtypes = [vp]
        L.dgamr_pool_bytes.argtypes = [vp, sz, sz]
        L.dgamr_pool_admit.argtypes = [vp, vp, ctypes.c_double, i32p, i64p, vp]
        L.dgamr_pool_release.argtypes = [vp, i32, vp]
        L.dgamr_pool_step.argtypes = [vp, vp, vp, vp]
        L.dgamr_pool_dt.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.dgamr_pool_stats.argtypes = [vp, i64p, i32p]
        L.dgamr_pool_set_shape.argtypes = [vp, i32, i32]
        L.dgamr_pool_set_lanes.argtypes = [vp, i32]
        L.dgamr_pool_autotune.argtypes = [vp, vp, vp, vp, i32p, i32p, i32p, ctypes.POINTER(ctypes.c_double)]
        L.dgamr_pools_capture.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, i32,
                                          ctypes.POINTER(vp)]
        L.dgamr_graph_launch.argtypes = [vp, vp]
        L.dgamr_graph_destroy.argtypes = [vp]
        L.dgamr_run_capture.argtypes = [vp, ctypes.c_double, ctypes.c_int, vp, vp, vp, ctypes.POINTER(vp)]
        L.dgamr_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "dgamr_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise DgamrError(rc, lib().dgamr_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def check_buffer(t, name, dtype, numel, at_least=False, device_type="cuda"):
    """Raise ValueError unless `t` is a contiguous torch tensor of `dtype`
    with `numel` elements (at least `numel` when at_least) on the GPU.  The
    C-ABI receives bare device pointers without sizes, so a stale or
    mistyped buffer would be written past its end by the kernels; this is
    the check that keeps it a Python error."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: the tensor must be contiguous")
    n = t.numel()
    if (n < numel) if at_least else (n != numel):
        raise ValueError(f"{name}: {n} elements, expected {'at least ' if at_least else ''}{numel} "
                         "(sized for another forest, or for this forest before a refinement?)")
    if t.device.type != device_type:
        raise ValueError(f"{name}: on {t.device}, expected a {device_type} device tensor")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def math_probe(fn: int, x, stream=None):
    """The stage kernels' FP64 reciprocal (fn 0) or square root (fn 1) of a
    device tensor (dgamr_math_probe)."""
    check_buffer(x, "x", torch.float64, x.numel())
    y = torch.empty_like(x)
    _check(lib().dgamr_math_probe(fn, _ptr(x), _ptr(y), x.numel(), _stream(stream)))
    return y


class Forest:
    """A device-resident forest of DG blocks (``dgamr_forest``)."""

    def __init__(self, dim, degree, n_cell, roots, lo, hi, bc, max_level, gamma=1.4,
                 precision=FP64, hanging=HANG_PAPER, limiter=LIMITER_NONE, equation=EQ_EULER,
                 velocity=(1.0, 1.0, 1.0), nu=1.0, exact_a=(-1.0, 1.0, 0.0)):
        d = ForestDesc()
        d.dim, d.degree, d.n_cell = dim, degree, n_cell
        roots, lo, hi, bc = (list(x) for x in (roots, lo, hi, bc))
        for a in range(3):
            d.roots[a] = roots[a] if a < dim else 1
            d.lo[a] = lo[a] if a < dim else 0.0
            d.hi[a] = hi[a] if a < dim else 1.0
            d.bc[a] = bc[a] if a < dim else BC_PERIODIC
        d.max_level, d.gamma = max_level, gamma
        d.precision, d.hanging, d.limiter = precision, hanging, limiter
        d.equation = equation
        for a in range(3):
            d.velocity[a] = velocity[a] if a < len(velocity) else 0.0
            d.exact_a[a] = exact_a[a] if a < len(exact_a) else 0.0
        d.diffusivity = nu
        self.desc = d
        self.dim, self.degree, self.N = dim, degree, n_cell
        self.equation = equation
        self.nv = 1 if equation in (EQ_ADVECTION, EQ_DIFFUSION) else dim + 2
        self.nb = {2: [1, 3, 6, 10], 3: [1, 4, 10, 20]}[dim][degree]
        self.precision = precision
        h = ctypes.c_void_p()
        _check(lib().dgamr_create_forest(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self._planned = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgamr_destroy_forest(self.h)
            self.h = None

    # ---- queries
    @property
    def n_leaves(self) -> int:
        n = ctypes.c_int64()
        _check(lib().dgamr_num_leaves(self.h, ctypes.byref(n)))
        return n.value

    @property
    def ncell(self) -> int:
        return self.N ** self.dim

    @property
    def time(self) -> float:
        """Time of the state (the Dirichlet data of a diffusion forest)."""
        t = ctypes.c_double()
        _check(lib().dgamr_get_time(self.h, ctypes.byref(t)))
        return t.value

    @time.setter
    def time(self, t: float):
        _check(lib().dgamr_set_time(self.h, t))

    def set_root_frames(self, codes):
        """Rotation code of each root's local frame (dgamr_set_root_frames)."""
        c = torch.as_tensor(list(codes), dtype=torch.int32).contiguous()
        if c.numel() != self.desc.roots[0] * self.desc.roots[1] * self.desc.roots[2]:
            raise ValueError("one frame code per root")
        _check(lib().dgamr_set_root_frames(self.h, _ptr(c)))

    def set_root_nodes(self, xy):
        """Bilinear (3-D: trilinear) root blocks from the root grid nodes,
        shape (roots_y + 1, roots_x + 1, 2) or (roots_z + 1, roots_y + 1,
        roots_x + 1, 3) (dgamr_set_root_nodes)."""
        a = torch.as_tensor(xy, dtype=torch.float64).contiguous()
        d = self.desc.dim
        n = (self.desc.roots[0] + 1) * (self.desc.roots[1] + 1) * (self.desc.roots[2] + 1 if d == 3 else 1)
        if a.numel() != d * n:
            raise ValueError("one node of dim coordinates per root grid vertex")
        _check(lib().dgamr_set_root_nodes(self.h, _ptr(a)))

    def keys(self):
        k = torch.zeros((self.n_leaves, 5), dtype=torch.int32)
        _check(lib().dgamr_leaf_keys(self.h, _ptr(k)))
        return k.numpy()

    def sizes(self):
        u, g, r, w = (ctypes.c_size_t() for _ in range(4))
        _check(lib().dgamr_state_bytes(self.h, ctypes.byref(u), ctypes.byref(g), ctypes.byref(r), ctypes.byref(w)))
        return u.value, g.value, r.value, w.value

    # ---- allocation helpers (caller-owned device buffers)
    def state_shape(self):
        return (self.n_leaves, self.nv, self.nb, self.ncell)

    def guard_shape(self):
        return (self.n_leaves, 2 * self.dim, self.nv, self.nb, self.N ** (self.dim - 1))

    def new_state(self, device="cuda"):
        return torch.zeros(self.state_shape(), dtype=torch.float64, device=device)

    def new_guard(self, device="cuda"):
        return torch.zeros(self.guard_shape(), dtype=torch.float64, device=device)

    def new_residual(self, device="cuda"):
        dt = torch.float32 if self.precision == FP32 else torch.float64
        return torch.zeros(self.state_shape(), dtype=dt, device=device)

    def new_work(self, device="cuda"):
        return torch.zeros(self.sizes()[3] // 8, dtype=torch.float64, device=device)

    # ---- buffer checks (the C-ABI takes bare pointers)
    def _state_elems(self):
        return self.n_leaves * self.nv * self.nb * self.ncell

    def _chk_state(self, t, name="u"):
        check_buffer(t, name, torch.float64, self._state_elems())

    def _chk_guard(self, t, name="guard"):
        check_buffer(t, name, torch.float64, self.sizes()[1] // 8)

    def _chk_res(self, t, name="r"):
        dt = torch.float32 if self.precision == FP32 else torch.float64
        check_buffer(t, name, dt, self._state_elems())

    def _chk_work(self, t, name="work"):
        check_buffer(t, name, torch.float64, (self.sizes()[3] + 7) // 8, at_least=True)

    def _chk_dt(self, t, name="dt_dev"):
        check_buffer(t, name, torch.float64, 1, at_least=True)

    # ---- C-ABI calls
    def set_refinement(self, flags) -> int:
        f = torch.as_tensor(flags, dtype=torch.int8).contiguous()
        if f.numel() != self.n_leaves:
            raise ValueError(f"flags: {f.numel()} entries for {self.n_leaves} leaves")
        n = ctypes.c_int64()
        _check(lib().dgamr_set_refinement(self.h, _ptr(f), ctypes.byref(n)))
        self._planned = n.value
        return n.value

    def apply_refinement(self, u_old, u_new, stream=None):
        """u_new: caller-allocated state of the size set_refinement returned."""
        self._chk_state(u_old, "u_old")
        if self._planned is None:
            raise ValueError("apply_refinement: no refinement plan pending (call set_refinement first)")
        check_buffer(u_new, "u_new", torch.float64, self._planned * self.nv * self.nb * self.ncell)
        self._planned = None
        _check(lib().dgamr_apply_refinement(self.h, _ptr(u_old), _ptr(u_new), _stream(stream)))

    def adapt(self, flags, u_old, stream=None):
        """set_refinement + apply_refinement; returns the new state tensor."""
        n_new = self.set_refinement(flags)
        u_new = torch.zeros((n_new, self.nv, self.nb, self.ncell), dtype=torch.float64, device=u_old.device)
        self.apply_refinement(u_old, u_new, stream)
        return u_new

    def fill_guardcells(self, u, guard, stream=None):
        self._chk_state(u)
        self._chk_guard(guard)
        _check(lib().dgamr_fill_guardcells(self.h, _ptr(u), _ptr(guard), _stream(stream)))

    def dg_residual(self, u, guard, r, stream=None):
        self._chk_state(u)
        self._chk_guard(guard)
        self._chk_res(r)
        _check(lib().dgamr_dg_residual(self.h, _ptr(u), _ptr(guard), _ptr(r), _stream(stream)))

    def rk_stage(self, stage, dt_dev, u_n, u_s, r, u_next, stream=None):
        self._chk_dt(dt_dev)
        if stage > 0:
            self._chk_state(u_n, "u_n")
        self._chk_state(u_s, "u_s")
        self._chk_res(r)
        self._chk_state(u_next, "u_next")
        _check(lib().dgamr_rk_stage(self.h, stage, _ptr(dt_dev), _ptr(u_n), _ptr(u_s), _ptr(r), _ptr(u_next),
                                    _stream(stream)))

    def compute_dt(self, cfl, u, dt_dev, work, stream=None):
        self._chk_state(u)
        self._chk_dt(dt_dev)
        self._chk_work(work)
        _check(lib().dgamr_compute_dt(self.h, cfl, _ptr(u), _ptr(dt_dev), _ptr(work), _stream(stream)))

    def step(self, u, work, dt_dev, cfl=0.1, stream=None):
        """One SSP-RK3 step in place; cfl <= 0 uses the dt already in dt_dev."""
        self._chk_state(u)
        self._chk_work(work)
        self._chk_dt(dt_dev)
        _check(lib().dgamr_step(self.h, cfl, _ptr(u), _ptr(work), _ptr(dt_dev), _stream(stream)))

    def step_static(self, u, dt_dev, cfl=0.1, stream=None):
        """One SSP-RK3 step in place with the library's static work area
        (dgamr_step_static: allocates nothing)."""
        self._chk_state(u)
        self._chk_dt(dt_dev)
        _check(lib().dgamr_step_static(self.h, cfl, _ptr(u), _ptr(dt_dev), _stream(stream)))

    def run(self, u, work, dt_dev, nsteps, cfl=0.1, stream=None):
        """nsteps SSP-RK3 steps in place, three launches per step."""
        self._chk_state(u)
        self._chk_work(work)
        self._chk_dt(dt_dev)
        _check(lib().dgamr_run(self.h, cfl, nsteps, _ptr(u), _ptr(work), _ptr(dt_dev), _stream(stream)))

    def capture_run(self, u, work, dt_dev, nsteps, cfl=0.1):
        """nsteps steps of run() captured into a HIP graph (RunGraph); each
        launch advances u by nsteps steps."""
        self._chk_state(u)
        self._chk_work(work)
        self._chk_dt(dt_dev)
        h = ctypes.c_void_p()
        _check(lib().dgamr_run_capture(self.h, cfl, nsteps, _ptr(u), _ptr(work), _ptr(dt_dev), ctypes.byref(h)))
        return RunGraph(h, keep=(self, u, work, dt_dev))

    def conserved_totals(self, u, work, stream=None):
        self._chk_state(u)
        self._chk_work(work)
        t = torch.zeros(self.nv, dtype=torch.float64, device=u.device)
        _check(lib().dgamr_conserved_totals(self.h, _ptr(u), _ptr(t), _ptr(work), _stream(stream)))
        return t

    def limit_positivity(self, u, stream=None):
        self._chk_state(u)
        _check(lib().dgamr_limit_positivity(self.h, _ptr(u), _stream(stream)))

    def indicator(self, u, work, stream=None):
        self._chk_state(u)
        self._chk_work(work)
        eta = torch.zeros(self.n_leaves, dtype=torch.float64, device=u.device)
        _check(lib().dgamr_indicator(self.h, _ptr(u), _ptr(eta), _ptr(work), _stream(stream)))
        return eta

    def project_ic(self, kind, params, t=0.0, u=None, stream=None):
        if u is None:
            u = self.new_state()
        self._chk_state(u)
        prm = (ctypes.c_double * 8)(*(list(params) + [0.0] * (8 - len(params))))
        _check(lib().dgamr_project_ic(self.h, kind, prm, t, _ptr(u), _stream(stream)))
        return u

    def check_state(self, u, work, stream=None) -> int:
        self._chk_state(u)
        self._chk_work(work)
        bad = ctypes.c_int64()
        rc = lib().dgamr_check_state(self.h, _ptr(u), ctypes.byref(bad), _ptr(work), _stream(stream))
        if rc not in (OK, ENONPHYSICAL):
            _check(rc)
        return bad.value

    def set_tuning(self, knob, value):
        _check(lib().dgamr_set_tuning(self.h, knob, value))

    def profile_enable(self, enable=True):
        _check(lib().dgamr_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self):
        """(summed stage-kernel milliseconds, launches) since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().dgamr_profile_read(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Pool:
    """Arena of leaf slots for many forests of one class (``dgamr_pool``),
    stepped together; the state arena and work buffer are owned here as
    torch tensors."""

    def __init__(self, dim, degree, n_cell, capacity_leaves, max_members, gamma=1.4, precision=FP64,
                 hanging=HANG_PAPER, limiter=LIMITER_NONE, device="cuda"):
        d = ForestDesc()
        d.dim, d.degree, d.n_cell, d.max_level, d.gamma = dim, degree, n_cell, 1, gamma
        for a in range(3):
            d.roots[a], d.lo[a], d.hi[a], d.bc[a] = 1, 0.0, 1.0, BC_PERIODIC
        d.precision, d.hanging, d.limiter = precision, hanging, limiter
        self.desc = d
        self.dim, self.degree, self.N = dim, degree, n_cell
        self.nv = dim + 2
        self.nb = {2: [1, 3, 6, 10], 3: [1, 4, 10, 20]}[dim][degree]
        self.ncell = n_cell ** dim
        self.capacity, self.max_members = capacity_leaves, max_members
        h = ctypes.c_void_p()
        _check(lib().dgamr_pool_create(ctypes.byref(d), capacity_leaves, max_members, ctypes.byref(h)))
        self.h = h
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().dgamr_pool_bytes(self.h, ctypes.byref(sb), ctypes.byref(wb)))
        self.state_bytes, self.work_bytes = sb.value, wb.value
        self.u = torch.zeros((capacity_leaves, self.nv, self.nb, self.ncell), dtype=torch.float64, device=device)
        self.work = torch.zeros(wb.value // 8, dtype=torch.float64, device=device)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            try:
                torch.cuda.synchronize()
            except Exception:
                pass
            _lib.dgamr_pool_destroy(self.h)
            self.h = None

    def leaf_bytes(self) -> int:
        return 8 * self.nv * self.nb * self.ncell

    def admit(self, forest: Forest, cfl: float, stream=None):
        """Admit a forest; returns (member id, first slot).  Raises
        DgamrError with code EFULL when it does not fit."""
        m, first = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().dgamr_pool_admit(self.h, forest.h, cfl, ctypes.byref(m), ctypes.byref(first),
                                      _stream(stream)))
        return m.value, first.value

    def release(self, member: int, stream=None):
        _check(lib().dgamr_pool_release(self.h, member, _stream(stream)))

    def view(self, first: int, n_leaves: int):
        """The member's state: a view of the arena at its slot range."""
        return self.u[first:first + n_leaves]

    def step(self, stream=None):
        _check(lib().dgamr_pool_step(self.h, _ptr(self.u), _ptr(self.work), _stream(stream)))

    def dt(self):
        """Per-member dt of the last step (device tensor view)."""
        p = ctypes.c_void_p()
        _check(lib().dgamr_pool_dt(self.h, _ptr(self.work), ctypes.byref(p)))
        off = (p.value - self.work.data_ptr()) // 8
        return self.work[off:off + self.max_members]

    def stats(self):
        n, m = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().dgamr_pool_stats(self.h, ctypes.byref(n), ctypes.byref(m)))
        return n.value, m.value

    def set_shape(self, rows=0, grid=0):
        _check(lib().dgamr_pool_set_shape(self.h, rows, grid))

    def set_lanes(self, rows=0):
        """The lane-per-(cell, variable) stage kernel with slabs of `rows`."""
        _check(lib().dgamr_pool_set_lanes(self.h, rows))

    def autotune(self, stream=None):
        """Returns (variant, rows, grid, best stage-launch microseconds);
        variant 1 = one thread per cell, 0 = one lane per (cell, variable)."""
        v, r, g, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().dgamr_pool_autotune(self.h, _ptr(self.u), _ptr(self.work), _stream(stream), ctypes.byref(v),
                                         ctypes.byref(r), ctypes.byref(g), ctypes.byref(us)))
        return v.value, r.value, g.value, us.value


class RunGraph:
    """A captured HIP graph (``dgamr_graph``); keeps what it references
    alive."""

    def __init__(self, h, keep=()):
        self.h = h
        self.keep = keep

    def launch(self, stream=None):
        _check(lib().dgamr_graph_launch(self.h, _stream(stream)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgamr_graph_destroy(self.h)
            self.h = None


class Graph(RunGraph):
    """HIP graph of nsteps steps of several pools (``dgamr_pools_capture``)."""

    def __init__(self, pools, nsteps: int):
        n = len(pools)
        hp = (ctypes.c_void_p * n)(*[p.h for p in pools])
        up = (ctypes.c_void_p * n)(*[p.u.data_ptr() for p in pools])
        wp = (ctypes.c_void_p * n)(*[p.work.data_ptr() for p in pools])
        h = ctypes.c_void_p()
        _check(lib().dgamr_pools_capture(hp, up, wp, n, nsteps, ctypes.byref(h)))
        super().__init__(h, keep=list(pools))  # keep the pools alive while the graph exists
