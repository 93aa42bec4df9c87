"""Observed order of accuracy of the GPU path, FP64 and FP32 residual: the
isentropic vortex advected on a 4x4-root periodic forest (8^2 and 16^2
cells per block: 32 and 64 cells across the period), L2 error of the
density against the exact translated vortex (evaluated by the oracle's
error norm on the GPU state).  Both precisions show order p + 1.  The
FP32 residual changes the error by at most 1 % plus 2e-6: its rounding
(unit roundoff 6e-8 on an O(1) state, accumulated over O(100) stages at
O(1e-2) dt) stays far below the truncation error."""
import math

import numpy as np
import pytest

import oracle as O
from tests.test_oracle_solver import VORTEX_20

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu_error(p, N, T, precision):
    from paper_2502_12620_amd import dgamr as G

    f = G.Forest(2, p, N, (4, 4), (0.0, 0.0), (20.0, 20.0), (0, 0), 2, precision=precision)
    u = f.project_ic(G.IC_VORTEX, VORTEX_20)
    h = 5.0 / N
    dt0 = 0.05 * h if p < 3 else 0.05 * h ** (4.0 / 3.0)
    n = int(math.ceil(T / dt0))
    work = f.new_work()
    dt = torch.full((1,), T / n, dtype=torch.float64, device="cuda")
    for _ in range(n):
        f.step(u, work, dt, 0.0)  # fixed dt
    torch.cuda.synchronize()
    orc = O.Forest(2, p, N, (4, 4), (0.0, 0.0), (20.0, 20.0), (0, 0), 2)
    return orc.errors(np.ascontiguousarray(u.cpu().numpy()), O.IC_VORTEX, VORTEX_20, T)[1][0]


@pytest.mark.parametrize("p,Ns,T", [(1, (8, 16), 1.0), (2, (8, 16), 1.0), (3, (8, 16), 0.5)])
def test_vortex_order_fp64_and_fp32(p, Ns, T):
    from paper_2502_12620_amd import dgamr as G

    e64 = [_gpu_error(p, N, T, G.FP64) for N in Ns]
    e32 = [_gpu_error(p, N, T, G.FP32) for N in Ns]
    for errs in (e64, e32):
        order = math.log2(errs[0] / errs[1])
        assert order >= p + 1 - 0.3, (errs, order)
    for a, b in zip(e32, e64):
        assert abs(a - b) <= 1e-2 * b + 2e-6, (e32, e64)
    print(f"p={p}: L2 fp64 {e64}, fp32 {e32}, order {math.log2(e64[0] / e64[1]):.2f} / "
          f"{math.log2(e32[0] / e32[1]):.2f}")
