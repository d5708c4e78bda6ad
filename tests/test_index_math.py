"""Neighbour addressing of the AA-pattern step kernels, checked on the CPU.

The odd step reads and writes the populations of the 3 x 3 neighbourhood in
the blocked layout (64-node blocks, populations contiguous per block).  The
kernels form those element offsets with 32-bit node arithmetic (one 64-bit
product per row); `tests/native/nbr_check.hip` compiles the same device
header for the host and compares every offset with the plain 64-bit index of
the wrapped neighbour node, on ragged grids (all nodes), a 4096^2 grid, the
largest grid and the widest grid the library accepts (edge rows and columns),
for m = 1..4; likewise the 3-D path's offsets (ragged boxes, 256^3, the
largest and the widest boxes).  The limits themselves are checked through lb_init validation.
"""
import os
import shutil
import subprocess

import pytest

from paper_2101_03055_amd import lb, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not found")


def test_neighbour_offsets_match_blocked_index(tmp_path):
    exe = str(tmp_path / "nbr_check")
    subprocess.check_call([hipcc(), "--offload-arch=gfx950", "-O2", "-std=c++20",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           f"-I{os.path.join(ROOT, 'include')}",
                           f"-I{os.path.join(ROOT, 'paper_2101_03055_amd', 'csrc')}",
                           os.path.join(ROOT, "tests", "native", "nbr_check.hip"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:]
    assert "all neighbour offsets agree" in out.stdout
    assert out.stdout.count("ok M=") == 4 * 13
    assert out.stdout.count("ok 3-D M=") == 4 * 10


@pytest.mark.parametrize("m,nx,ok", [(2, 2 ** 31 // 19 - 64 - 1, True), (2, 2 ** 31 // 19 - 64 + 1, False),
                                     (4, 2 ** 31 // 29 - 64 - 1, True), (4, 2 ** 31 // 29 - 64 + 1, False)])
def test_width_limit(m, nx, ok):
    wl, _, _, _ = W.random_case(8, 8, m=m, seed=1)
    p = lb.params_from_workload(wl, "f64")
    p.nx = nx
    p.ny = 2
    if ok:
        assert lb.lb_workspace_bytes(p) > 0
    else:
        with pytest.raises(lb.LBError) as ei:
            lb.lb_workspace_bytes(p)
        assert "wide" in str(ei.value)
