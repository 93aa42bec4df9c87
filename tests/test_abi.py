"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/dgamr.h declares, and rejects bad descriptors with the
documented error codes before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgamr.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dgamr_[a-z_]+)\s*\(", txt)))


def _lib():
    from paper_2502_12620_amd import dgamr as G

    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libdgamr.so not built")
    return G, G.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("dgamr_create_forest", "dgamr_set_refinement", "dgamr_fill_guardcells",
                     "dgamr_dg_residual", "dgamr_rk_stage", "dgamr_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    G, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(G.EXPORTS) == set(_declared())


def _desc(G, **kw):
    d = G.ForestDesc()
    d.dim, d.degree, d.n_cell = kw.get("dim", 2), kw.get("degree", 1), kw.get("n_cell", 8)
    for a in range(3):
        d.roots[a] = 1
        d.lo[a] = 0.0
        d.hi[a] = 1.0
        d.bc[a] = 0
    d.max_level = kw.get("max_level", 1)
    d.gamma = kw.get("gamma", 1.4)
    d.precision = kw.get("precision", 0)
    d.hanging = kw.get("hanging", 0)
    d.limiter = kw.get("limiter", 0)
    return d


@pytest.mark.parametrize("bad,code", [
    (dict(dim=4), -1), (dict(degree=4), -2), (dict(n_cell=7), -1), (dict(n_cell=0), -1),
    (dict(n_cell=18), -2), (dict(dim=3, n_cell=10), -2), (dict(max_level=0), -1), (dict(gamma=1.0), -1),
    (dict(precision=7), -1), (dict(hanging=3), -1), (dict(limiter=2), -1),
])
def test_bad_descriptors_are_rejected(bad, code):
    G, L = _lib()
    h = ctypes.c_void_p()
    rc = L.dgamr_create_forest(ctypes.byref(_desc(G, **bad)), ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert len(L.dgamr_last_error()) > 0


def test_null_arguments_are_rejected():
    G, L = _lib()
    assert L.dgamr_create_forest(None, None) == G.EINVAL
    assert L.dgamr_num_leaves(None, None) == G.EINVAL
    assert L.dgamr_step(None, ctypes.c_double(0.1), None, None, None, None) == G.EINVAL
    assert b"null" in L.dgamr_last_error()


def test_pool_and_graph_arguments_are_checked_before_any_device_call():
    G, L = _lib()
    h = ctypes.c_void_p()
    assert L.dgamr_pool_create(None, 16, 4, ctypes.byref(h)) == G.EINVAL
    d = _desc(G)
    assert L.dgamr_pool_create(ctypes.byref(d), 0, 4, ctypes.byref(h)) == G.EINVAL
    assert L.dgamr_pool_create(ctypes.byref(d), 16, 0, ctypes.byref(h)) == G.EINVAL
    assert L.dgamr_pool_create(ctypes.byref(_desc(G, n_cell=7)), 16, 4, ctypes.byref(h)) == G.EINVAL
    assert not h.value
    assert L.dgamr_pool_step(None, None, None, None) == G.EINVAL
    assert L.dgamr_pool_set_lanes(None, 0) == G.EINVAL
    assert L.dgamr_pool_admit(None, None, ctypes.c_double(0.1), None, None, None) == G.EINVAL
    assert L.dgamr_pool_release(None, 0, None) == G.EINVAL
    assert L.dgamr_graph_launch(None, None) == G.EINVAL
    assert L.dgamr_run_capture(None, ctypes.c_double(0.1), 1, None, None, None, None) == G.EINVAL
    assert L.dgamr_pool_destroy(None) == G.OK
    assert L.dgamr_graph_destroy(None) == G.OK


def test_binding_buffer_checks_on_the_host():
    """The binding's buffer check (the C-ABI takes bare pointers) refuses a
    wrong dtype, a non-contiguous view, a stale size and a host tensor, in
    that order, before anything reaches the library."""
    torch = pytest.importorskip("torch")
    from paper_2502_12620_amd import dgamr as G

    t = torch.zeros(12, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        G.check_buffer(t.float(), "u", torch.float64, 12)
    with pytest.raises(ValueError, match="contiguous"):
        G.check_buffer(torch.zeros(4, 6, dtype=torch.float64).t(), "u", torch.float64, 24)
    with pytest.raises(ValueError, match="13"):
        G.check_buffer(t, "u", torch.float64, 13)
    with pytest.raises(ValueError, match="at least 20"):
        G.check_buffer(t, "work", torch.float64, 20, at_least=True)
    with pytest.raises(ValueError, match="device"):
        G.check_buffer(t, "u", torch.float64, 12)
    G.check_buffer(t, "u", torch.float64, 12, device_type="cpu")
    G.check_buffer(t, "work", torch.float64, 8, at_least=True, device_type="cpu")
