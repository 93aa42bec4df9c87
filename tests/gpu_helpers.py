"""Helpers for the GPU parity tests: build the oracle forest and the GPU
forest of one workload side by side and compare states by leaf key."""
import numpy as np

import oracle as O
from paper_2502_12620_amd import workloads as W


def make_pair(w, hanging=0, limiter=False, precision=None):
    import torch  # noqa: F401
    from paper_2502_12620_amd import dgamr as G

    orc = O.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma, hanging=hanging)
    gpu = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma,
                   precision=G.FP64 if precision is None else precision, hanging=hanging,
                   limiter=G.LIMITER_POSITIVITY if limiter else G.LIMITER_NONE)
    import torch

    for rule in w.initial_refinement:
        orc.adapt(rule(w, orc.keys()))
        gpu.adapt(rule(w, gpu.keys()), torch.zeros(gpu.state_shape(), dtype=torch.float64, device="cuda"))
    assert np.array_equal(orc.keys(), gpu.keys()), "leaf keys differ"
    return orc, gpu


def rel_diff(got, ref):
    """Per-variable max |got - ref| / max |ref| over all coefficients."""
    nv = ref.shape[1]
    out = []
    for v in range(nv):
        scale = np.abs(ref[:, v]).max()
        out.append(np.abs(got[:, v] - ref[:, v]).max() / (scale if scale > 0 else 1.0))
    return np.array(out)


def rel_diff_floored(got, ref, floor=1e-6):
    """rel_diff with each variable's scale floored at floor x the largest
    coefficient (for variables that are zero up to rounding, such as the z
    momentum of an extruded vortex)."""
    big = np.abs(ref).max()
    out = []
    for v in range(ref.shape[1]):
        scale = max(np.abs(ref[:, v]).max(), floor * big)
        out.append(np.abs(got[:, v] - ref[:, v]).max() / (scale if scale > 0 else 1.0))
    return np.array(out)


def small_c2(n_cell=4):
    """The two-level vortex forest of the 2-D AMR workload at a smaller block
    size, for runs the oracle finishes in seconds."""
    w = W.vortex_c2()
    w.n_cell = n_cell
    return w
