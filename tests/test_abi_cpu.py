"""Host-side checks of the C-ABI library (no GPU needed).

* libamrv.so loads and exports every function include/amrv.h declares;
* the host forest validation (called by amrv_workspace_bytes) accepts the
  workload forests and rejects unbalanced / non-covering ones, like the oracle.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2004_03275_amd import _native as N
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared():
    txt = "".join(open(h).read() for h in HEADERS)
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(amrv_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libamrv.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (amrv_\w+)", out))
    declared = _declared()
    assert declared, "no declarations parsed"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    # and the binding knows every one of them with a signature
    assert set(declared) == set(N.SIGNATURES), set(declared) ^ set(N.SIGNATURES)
    N.lib()  # loads without a GPU


def _ws(forest):
    cfg = N.make_config(forest.scheme)
    lev = np.ascontiguousarray(forest.level, np.int32)
    ijk = np.ascontiguousarray(forest.ijk, np.int32)
    n = N.lib().amrv_workspace_bytes(ctypes.byref(cfg), forest.n, lev.ctypes.data, ijk.ctypes.data)
    return n, N.lib().amrv_last_error().decode()


@pytest.mark.parametrize("which", ["sod", "kh", "ot"])
def test_workspace_for_uniform_workloads(which):
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libamrv.so not built")
    f = {"sod": lambda: W.sod()[0], "kh": lambda: W.kh(4)[0], "ot": lambda: W.orszag_tang(4)[0]}[which]()
    n, err = _ws(f)
    state = f.scheme.nvar * f.n * f.scheme.cells_per_block * 8
    assert n >= 3 * state, err


def test_host_validation_matches_oracle_contract():
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libamrv.so not built")
    s = W.Scheme(ndim=2, block_nx=(16, 16), base_blocks=(2, 2), max_level=3)
    lev = [1, 1, 1] + [3] * 4 + [2] * 3
    ijk = [[1, 0, 0], [0, 1, 0], [1, 1, 0]] + [[a & 1, a >> 1, 0] for a in range(4)] + [[1, 0, 0], [0, 1, 0], [1, 1, 0]]
    f = W.Forest(s, np.array(lev, np.int32), np.array(ijk, np.int32))
    n, err = _ws(f)
    assert n == 0 and "balance" in err
    gap = W.Forest(s, np.array([1, 1, 1], np.int32), np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.int32))
    n, err = _ws(gap)
    assert n == 0 and "cover" in err
    s3 = W.Scheme(ndim=3, block_nx=(8, 8, 8), base_blocks=(2, 2, 2))
    n, err = _ws(W.uniform_forest(s3))
    assert n == 0 and "16-cell" in err


def test_blast_forest_tables_build():
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libamrv.so not built")
    s = W.blast_scheme(base=4, max_level=3)
    f = W.blast_forest(s, radius=0.1, buffer_cells=2)
    assert len(f.level_counts()) == 3
    n, err = _ws(f)
    assert n > 0, err


def test_workspace_holds_the_z_buffer_of_3d_mhd_only():
    """3D MHD forests carry one more state-sized buffer (the z flux divergence
    of the two-launch stage update); the same leaves with Euler do not."""
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libamrv.so not built")
    f, _ = W.mhd_blast(3, scheme=W.mhd_blast_scheme(3, base=2, max_level=2))
    n_mhd, err = _ws(f)
    assert n_mhd > 0, err
    state = f.scheme.nvar * f.n * f.scheme.cells_per_block * 8
    assert n_mhd >= 4 * state
    f2, _ = W.mhd_blast(2, scheme=W.mhd_blast_scheme(2, base=2, max_level=2))
    n2, err = _ws(f2)
    state2 = f2.scheme.nvar * f2.n * f2.scheme.cells_per_block * 8
    assert 3 * state2 <= n2 < 4 * state2, err
