"""Host side of the forest Helmholtz solver (amrv_fmg_*): the block tree's
validation and workspace size, without a GPU."""
import os

import numpy as np
import pytest

import workloads as W
from paper_2004_03275_amd import _native as N
from paper_2004_03275_amd import multigrid as MG

pytestmark = pytest.mark.skipif(not os.path.exists(N.LIB_PATH), reason="libamrv.so not built")


def _forest(base=4, max_level=3, bc=W.PERIODIC):
    return W.fmg_forest(W.fmg_scheme(base=base, max_level=max_level, bc=bc), centre=(0.27, 0.3), radius=0.15)


@pytest.mark.parametrize("bc", [MG.PERIODIC, MG.NEUMANN])
def test_workspace_covers_every_block_of_the_tree(bc):
    f = _forest(bc=bc)
    nbytes = MG.fmg_workspace_bytes(f, 1.0, bc)
    # leaves plus their ancestors, four block arrays of 256 doubles each
    anc = set()
    for l, i, j in zip(f.level, f.ijk[:, 0], f.ijk[:, 1]):
        while l > 1:
            l, i, j = l - 1, i >> 1, j >> 1
            anc.add((int(l), int(i), int(j)))
    assert nbytes >= (f.n + len(anc)) * 4 * 256 * 8


def _expect_error(forest, code=N.EUNBALANCED):
    with pytest.raises(N.AmrvError) as e:
        MG.fmg_workspace_bytes(forest, 1.0, MG.PERIODIC)
    assert e.value.code == code, e.value


def test_rejects_overlap_gap_and_imbalance():
    s = W.fmg_scheme(base=4, max_level=3)
    f = W.uniform_forest(s, level=1)
    # overlap: a level-2 child of block (0, 0) added to the level-1 leaves
    _expect_error(W.Forest(s, np.append(f.level, 2).astype(np.int32), np.vstack([f.ijk, [0, 0, 0]]).astype(np.int32)))
    # gap: one level-1 leaf missing
    _expect_error(W.Forest(s, f.level[1:].copy(), f.ijk[1:].copy()))
    # 2:1 balance: block (0, 0) refined twice, next to level-1 leaves
    lev, ijk = [], []
    for k in range(f.n):
        i, j = f.ijk[k, :2]
        if (i, j) != (0, 0):
            lev.append(1)
            ijk.append([i, j, 0])
    for a in range(2):
        for b in range(2):
            if (a, b) == (1, 1):
                for c in range(2):
                    for d in range(2):
                        lev.append(3)
                        ijk.append([2 + c, 2 + d, 0])
            else:
                lev.append(2)
                ijk.append([a, b, 0])
    _expect_error(W.Forest(s, np.array(lev, dtype=np.int32), np.array(ijk, dtype=np.int32)))


def test_rejects_bad_configuration():
    f = _forest()
    for field, value in (("base", 3), ("max_level", 0), ("pre_sweeps", 0), ("bc", 7)):
        cfg = MG.fmg_config(f, 1.0, MG.PERIODIC)
        setattr(cfg, field, value)
        lev = np.ascontiguousarray(f.level, dtype=np.int32)
        ijk = np.ascontiguousarray(f.ijk, dtype=np.int32)
        assert N.lib().amrv_fmg_workspace_bytes(cfg, lev.ctypes.data, ijk.ctypes.data) == 0, field


def test_3d_octree_forests():
    """Octree forests: the workspace covers every block of the tree; an
    octree that breaks 2:1 balance and a 3D base grid above 512 cells per
    side are rejected."""
    f = W.fmg_forest(W.fmg_scheme(base=2, max_level=3, bc=MG.NEUMANN, ndim=3), centre=(0.3, 0.35, 0.4), radius=0.15)
    nbytes = MG.fmg_workspace_bytes(f, 1.0, MG.NEUMANN)
    anc = set()
    for l, (i, j, k) in zip(f.level, f.ijk):
        while l > 1:
            l, i, j, k = l - 1, i >> 1, j >> 1, k >> 1
            anc.add((int(l), int(i), int(j), int(k)))
    assert nbytes >= (f.n + len(anc)) * 5 * 4096 * 8
    s = W.fmg_scheme(base=2, max_level=3, ndim=3)
    lev, ijk = [], []
    for k in range(2):
        for j in range(2):
            for i in range(2):
                if (i, j, k) != (0, 0, 0):
                    lev.append(1)
                    ijk.append([i, j, k])
    for q in range(8):
        a, b, c = q & 1, (q >> 1) & 1, q >> 2
        if q == 7:
            for r in range(8):
                lev.append(3)
                ijk.append([2 + (r & 1), 2 + ((r >> 1) & 1), 2 + (r >> 2)])
        else:
            lev.append(2)
            ijk.append([a, b, c])
    _expect_error(W.Forest(s, np.array(lev, dtype=np.int32), np.array(ijk, dtype=np.int32)))
    cfg = MG.fmg_config(f, 1.0, MG.PERIODIC)
    cfg.base = 64
    lev_a = np.ascontiguousarray(f.level, dtype=np.int32)
    ijk_a = np.ascontiguousarray(f.ijk, dtype=np.int32)
    assert N.lib().amrv_fmg_workspace_bytes(cfg, lev_a.ctypes.data, ijk_a.ctypes.data) == 0
