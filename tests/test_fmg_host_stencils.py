"""The forest multigrid's batched 3D stencils against its per-cell ones, on
the host: tests/host/fmg_stencils.hip includes csrc/fmg.hip, builds the
block tree of a forest and checks that stencil_k / apply_k (the loads of
four cells issued together, same-level neighbour blocks' cells folded into
the batch) give the sums of stencil / apply_cell bit for bit, for the plain
stencil on every block and the problem's rules (Sec. 1.4 coarse-fine faces)
on the leaves; the host side is built with AddressSanitizer, so every table
and neighbour access of those functions is bounds-checked too."""
import os
import shutil
import subprocess

import pytest

import workloads as W
from paper_2004_03275_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libamrv.so not built")
    lib = os.path.dirname(N.LIB_PATH)
    exe = str(tmp_path_factory.mktemp("fmgchk") / "fmg_stencils")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(lib, "csrc"), os.path.join(ROOT, "tests", "host", "fmg_stencils.hip"), "-L", lib, "-lamrv",
           f"-Wl,-rpath,{lib}", "-o", exe]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-3000:]
    return exe


CASES = [
    # ndim, base, max_level, centre, radius
    (3, 1, 3, (0.2, 0.2, 0.2), 0.1),
    (3, 1, 3, (0.3, 0.35, 0.4), 0.2),
    (2, 4, 3, (0.27, 0.3), 0.15),
    (2, 2, 4, (0.5, 0.45), 0.2),
]


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("nd,base,max_level,centre,radius", CASES)
def test_batched_stencils_equal_the_per_cell_ones(checker, tmp_path, bc, nd, base, max_level, centre, radius):
    f = W.fmg_forest(W.fmg_scheme(base=base, max_level=max_level, bc=bc, ndim=nd), centre=centre, radius=radius)
    assert f.n >= 1
    s = f.scheme
    path = tmp_path / "forest.txt"
    with open(path, "w") as fh:
        fh.write(f"{f.n} {s.base_blocks[0]} {s.max_level} {bc} {nd}\n")
        for k in range(f.n):
            fh.write(f"{f.level[k]} {f.ijk[k, 0]} {f.ijk[k, 1]} {f.ijk[k, 2]}\n")
    out = subprocess.run([checker, str(path)], capture_output=True, text=True, timeout=300)
    print(f.level_counts(), out.stdout.strip())
    assert out.returncode == 0, (out.stdout[-2000:], out.stderr[-3000:])
    assert "mismatches 0" in out.stdout
