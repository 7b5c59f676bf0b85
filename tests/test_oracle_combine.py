"""Pins of the oracle's submatrix combination (Sec. III-B, Eq.
combination_criterion) and of NOLSM on combined submatrices.

C1 a 5-molecule chain (N(J) = {J-1, J, J+1}) worked by hand: the pairs
   (0,1) and (3,4) pass the cubic criterion with nothing added to the larger
   side, (1,2) and (2,3) do not ((3+3-2)^3 = 64 > 27+27), so the groups are
   {0,1}, {2}, {3,4} and the cubic cost drops from 97 to 81 block^3.
C2 a block-diagonal pattern never merges ((1+1)^3 > 1+1).
C3 at termination no candidate pair passes the criterion within the cap,
   and the cubic cost never exceeds the uncombined one.
C4 full cell: every submatrix is the whole matrix, groups fill up to the cap,
   and D on the combined submatrices is still the exact C_occ C_occ^T.
C5 the trivial grouping (one molecule per group) reproduces the
   per-molecule oracle exactly.
"""
import numpy as np
import scipy.linalg as sla

import synth
from oracle import combine as cb
from oracle import nolsm as o


def chain(nb):
    ptr, blk = [0], []
    for J in range(nb):
        blk.extend(I for I in (J - 1, J, J + 1) if 0 <= I < nb)
        ptr.append(len(blk))
    return np.array(ptr), np.array(blk)


def groups_as_sets(g):
    grp_ptr, grp_blk, own_ptr, own_J = g
    return [sorted(own_J[own_ptr[i]:own_ptr[i + 1]].tolist()) for i in range(len(own_ptr) - 1)]


def test_c1_chain_by_hand():
    ptr, blk = chain(5)
    g = cb.combine_groups(5, ptr, blk)
    assert groups_as_sets(g) == [[0, 1], [2], [3, 4]]
    assert cb.cubic_cost(ptr) == 97.0
    assert cb.cubic_cost(g[0]) == 81.0
    grp_ptr, grp_blk = g[0], g[1]
    assert grp_blk[grp_ptr[0]:grp_ptr[1]].tolist() == [0, 1, 2]
    assert grp_blk[grp_ptr[2]:grp_ptr[3]].tolist() == [2, 3, 4]


def test_c2_block_diagonal_never_merges():
    ptr, blk = np.arange(9), np.arange(8)
    g = cb.combine_groups(8, ptr, blk)
    assert groups_as_sets(g) == [[J] for J in range(8)]


def test_c3_termination_and_cost(box64):
    s = box64
    plan = o.plan_arrays(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    g = cb.combine_groups(s.K.nb, plan["sub_ptr"], plan["sub_blk"])
    grp_ptr, grp_blk, own_ptr, own_J = g
    assert sorted(own_J.tolist()) == list(range(s.K.nb))
    assert cb.cubic_cost(grp_ptr) <= cb.cubic_cost(plan["sub_ptr"])
    rows = [set(grp_blk[grp_ptr[i]:grp_ptr[i + 1]].tolist()) for i in range(len(grp_ptr) - 1)]
    own = [set(own_J[own_ptr[i]:own_ptr[i + 1]].tolist()) for i in range(len(own_ptr) - 1)]
    for i in range(len(rows)):
        # a group's rows are the union of its molecules' N(J)
        union = set()
        for J in own[i]:
            union |= set(plan["sub_blk"][plan["sub_ptr"][J]:plan["sub_ptr"][J + 1]].tolist())
        assert rows[i] == union
        for j in range(len(rows)):
            if i == j or not (own[j] & rows[i]) or len(own[i]) + len(own[j]) > 10:
                continue
            mi, mj, mij = len(rows[i]), len(rows[j]), len(rows[i] & rows[j])
            assert not (mi + mj - mij) ** 3 < mi ** 3 + mj ** 3


def test_c4_full_cell_combined_is_exact():
    s = synth.water_cube(16, 0.7, config_id=102)
    assert s.K.nnzb == 16 * 16
    plan = o.plan_arrays(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    g = cb.combine_groups(s.K.nb, plan["sub_ptr"], plan["sub_blk"])
    assert [len(x) for x in groups_as_sets(g)] == [10, 6]
    r = o.nolsm_groups(s, g)
    assert np.all(r.status == o.OK)
    Kd, Sd = o.dense(s.K), o.dense(s.S)
    w, C = sla.eigh(Kd, Sd)
    Co = C[:, w < s.mu]
    Dex = Co @ Co.T
    D = o.dense_from_pattern(s.K.nb, s.K.bs, plan["D_row_ptr"], plan["D_col_idx"], r.D_val)
    assert np.linalg.norm(D - Dex) / np.linalg.norm(Dex) <= 1e-10
    assert abs(r.N.sum() - Co.shape[1]) < 1e-9


def test_c5_trivial_grouping_is_the_per_molecule_oracle(box64):
    s = box64
    plan = o.plan_arrays(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    nb = s.K.nb
    trivial = (plan["sub_ptr"], plan["sub_blk"], np.arange(nb + 1), np.arange(nb))
    a = o.nolsm(s, molecules=range(0, nb, 9))
    b = o.nolsm_groups(s, trivial)
    for J in range(0, nb, 9):
        assert np.allclose(b.Dcols[J], a.Dcols[J], rtol=0, atol=1e-13)
        assert abs(b.E[J] - a.E[J]) < 1e-12
