"""The FP64 reciprocal and square root of the stage kernels (Newton-Raphson
from the hardware reciprocal estimate; Goldschmidt plus one Newton
correction from the reciprocal-square-root estimate) against the correctly
rounded host results (IEEE division and square root) over wide ranges:
within one unit in the last place."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ulps(got, ref):
    return np.abs(got.view(np.int64) - ref.view(np.int64))


@pytest.mark.parametrize("fn", [0, 1])
def test_recip_and_sqrt_within_one_ulp(fn):
    from paper_2502_12620_amd import dgamr as G

    rng = np.random.default_rng(4 + fn)
    # magnitudes 1e-12 .. 1e12 (densities, gamma p / rho of near-vacuum and
    # blast states) plus values next to powers of two
    x = 10.0 ** rng.uniform(-12, 12, 2_000_000)
    edges = np.ldexp(1.0, np.arange(-40, 41))
    x = np.concatenate([x, edges, np.nextafter(edges, 0), np.nextafter(edges, np.inf)])
    y = G.math_probe(fn, torch.from_numpy(x).cuda()).cpu().numpy()
    ref = 1.0 / x if fn == 0 else np.sqrt(x)
    u = _ulps(y, ref)
    print(f"fn {fn}: max {u.max()} ulp, {np.mean(u > 0):.2e} of inputs not correctly rounded")
    assert u.max() <= 1


def test_sqrt_of_non_positive_is_zero():
    from paper_2502_12620_amd import dgamr as G

    x = torch.tensor([0.0, -1e-30, -1.0, -1e300], dtype=torch.float64, device="cuda")
    assert (G.math_probe(1, x).cpu() == 0).all()
