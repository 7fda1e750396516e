"""Leaf list of the 3D AMR blast built by Loehner refinement of its initial
state, with the oracle's estimator.

TEST INFRASTRUCTURE: this script writes an input fixture
(workloads/data/blast_lohner_forest.npz) from the oracle alone; the tests
check that the stored list is what it produces.

The paper refines a block by a fixed ratio of 2 as soon as one of its cells
has a Loehner error above the tolerance (Sec. 1.3).  Reading for the blast
workload: start from the level-1 grid of 16^3 blocks; at each level l below
the maximum, sample the initial state (p = 100 inside r < 0.1, 0.1 outside,
rho = 1, at rest) at the cell centres of the current forest, evaluate the
estimator on every level-l leaf, and refine every level-l leaf that has a
flagged cell within 8 cells (of level l, in every direction, periodic) of its
box: the block's own flagged cells plus an 8-cell buffer around those of its
neighbours.  2:1 balance across faces, edges and corners is restored after
each level (the workloads' forest builder), and the next level is evaluated
on the refined forest.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "workloads", "data", "blast_lohner_forest.npz")


def build(base: int = 16, max_level: int = 4, radius: float = 0.1, p_in: float = 100.0, p_out: float = 0.1,
          buffer_cells: int = 8, verbose: bool = False):
    """(level [n], ijk [n, 3]) of the Loehner-refined blast forest."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import oracle
    import workloads as W

    s = W.blast_scheme(base=base, max_level=max_level)
    nb0 = s.block_nx[0]
    tol = s.lohner_tol
    refine = set()  # (level, i, j, k) of every node refined so far
    forest = W.uniform_forest(s)
    for lev in range(1, max_level):
        _, U = W.blast(s, radius=radius, p_in=p_in, p_out=p_out, forest=forest)
        o = oracle.OracleForest(forest)
        o.set_state(U)
        _, emax = o.flag_blocks(with_emax=True)
        nblk = base << (lev - 1)
        marked = set()
        for b in np.nonzero((forest.level == lev) & (emax > tol))[0]:
            cells = o.lohner_cells(int(b))  # [z][y][x]
            loc = np.argwhere(cells > tol)[:, ::-1]  # (x, y, z) within the block
            g = forest.ijk[b].astype(np.int64) * nb0 + loc  # global cell indices at this level
            lo = np.floor_divide(g - buffer_cells, nb0)
            hi = np.floor_divide(g + buffer_cells, nb0)
            for a, c in zip(lo, hi):
                for i in range(a[0], c[0] + 1):
                    for j in range(a[1], c[1] + 1):
                        for k in range(a[2], c[2] + 1):
                            marked.add((lev, i % nblk, j % nblk, k % nblk))
        o.close()
        leaves = {(int(forest.level[b]), *map(int, forest.ijk[b])) for b in range(forest.n)}
        refine |= marked & leaves
        forest = W.refined_forest(s, lambda l, c: (l, *c) in refine)
        if verbose:
            print(f"level {lev}: {len(marked & leaves)} leaves flagged; forest {forest.n} leaves "
                  f"{forest.level_counts()}", flush=True)
    return forest.level.copy(), forest.ijk.copy()


def main():
    lev, ijk = build(verbose=True)
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    np.savez_compressed(OUT, level=lev.astype(np.int32), ijk=ijk.astype(np.int32))
    print(f"wrote {OUT}: {len(lev)} leaves")


if __name__ == "__main__":
    main()
