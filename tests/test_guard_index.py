"""The guard-cell source indices of the stage and fill kernels (which cell
of which neighbour block, and which child, feeds the guard cell at each face
point: Sec. 3.5, Eq. 15-17), compiled from the kernels' own header for the
host and checked against the forest's leaf geometry over random 2:1
refinements in 2-D and 3-D (tests/native/guard_index_check.cpp).  CPU only:
built with hipcc for the host."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_guard_cell_sources_match_the_geometry(tmp_path):
    exe = str(tmp_path / "guard_index_check")
    src = os.path.join(HERE, "native", "guard_index_check.cpp")
    forest = os.path.join(ROOT, "paper_2502_12620_amd", "csrc", "forest.cpp")
    cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fconstexpr-steps=200000000",
           "-I" + os.path.join(ROOT, "include"), src, forest, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1].startswith("OK")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_inline_combine_forms_agree_on_the_host(tmp_path):
    """The stage kernels' inline combine across hanging faces (children
    unrolled, zero table entries skipped) and the loop-over-children form
    that was withdrawn after a degree-3 GPU run gave NaN, both compiled for
    the host: bitwise equal on random states at degrees 1..3, 2-D and 3-D
    (tests/native/far_poly_forms.cpp)."""
    exe = str(tmp_path / "far_poly_forms")
    src = os.path.join(HERE, "native", "far_poly_forms.cpp")
    cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fconstexpr-steps=200000000",
           "-I" + os.path.join(ROOT, "include"), src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().splitlines()[-1].startswith("OK")
