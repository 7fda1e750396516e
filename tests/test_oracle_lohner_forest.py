"""The 3D AMR blast's leaf list (the stored input of the C4 workload) against
the Loehner refinement it stands for (no GPU).

The paper refines a block as soon as one of its cells has a Loehner error
above the tolerance (Sec. 1.3).  oracle/lohner_forest.py applies that rule
level by level to the blast's initial state with the oracle's estimator, an
8-cell buffer and 2:1 balance, and wrote workloads/data/blast_lohner_forest.npz.
"""
import numpy as np

import oracle
import workloads as W
from oracle import lohner_forest as LF


def _leafset(level, ijk):
    return set(zip(level.tolist(), map(tuple, ijk.tolist())))


def test_stored_forest_is_what_the_oracle_refinement_gives():
    s = W.blast_scheme()
    stored = W.blast_lohner_forest(s)
    lev, ijk = LF.build()
    assert np.array_equal(lev, stored.level) and np.array_equal(ijk, stored.ijk)
    assert stored.n == 19384
    assert stored.level_counts() == {1: 3888, 2: 1192, 3: 2272, 4: 12032}


def test_refinement_is_complete_and_balanced():
    """On the final forest no leaf below the top level has a flagged cell, and
    the oracle accepts the leaf list (cover, 2:1 balance)."""
    s = W.blast_scheme()
    f = W.blast_lohner_forest(s)
    _, U = W.blast(s, forest=f)
    o = oracle.OracleForest(f)
    o.set_state(U)
    _, emax = o.flag_blocks(with_emax=True)
    assert not np.any((emax > s.lohner_tol) & (f.level < s.max_level))
    assert np.sum(emax > s.lohner_tol) > 0  # the shell is flagged on the top level
    o.close()


def test_geometric_shell_forest_equals_the_loehner_forest():
    """The geometric generator (blocks whose box, grown by 8 cells, touches the
    sphere) gives the same leaves for this initial state."""
    s = W.blast_scheme()
    g = W.blast_forest(s)
    f = W.blast_lohner_forest(s)
    assert _leafset(g.level, g.ijk) == _leafset(f.level, f.ijk)
