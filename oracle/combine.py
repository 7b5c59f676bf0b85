"""Submatrix combination heuristic (Sec. III-B, 'Submatrix Combination
Heuristics', Eq. combination_criterion), plain Python.

TEST INFRASTRUCTURE ONLY: called by tests/, never by the library.

Groups start as one per molecule J, with row blocks R = N(J) and owned
molecules C = {J}. A group j is a merge candidate of group i when j owns a
block of R_i (the paper's first filter: rows of T_i). Merging i and j is
accepted iff the cubic cost drops (Eq. combination_criterion, in blocks; the
bs^3 factor cancels):

    (m_i + m_j - m_ij)^3 < m_i^3 + m_j^3,   m_ij = |R_i & R_j|.

Reading of the ordering: candidates are taken in increasing order of the
rows one side would add to the other, min(m_j - m_ij, m_i - m_ij) (the
paper's n_{j\\i}), one merge at a time; ties go to the larger drop
m_i^3 + m_j^3 - m_u^3, then to the smaller (min id, max id). The merged group
keeps the smaller id. A group owns at most `max_own` molecules (10: their
6-column unit blocks fill one 64-column tile). The heuristic stops when no
valid pair is left.
"""
from __future__ import annotations

import numpy as np


def combine_groups(nb, sub_ptr, sub_blk, max_own=10):
    """Returns (grp_ptr, grp_blk, own_ptr, own_J): group g has row blocks
    grp_blk[grp_ptr[g]:grp_ptr[g+1]] (sorted) and owns molecules
    own_J[own_ptr[g]:own_ptr[g+1]] (sorted); groups are ordered by their
    smallest owned molecule."""
    rows = {J: set(int(x) for x in sub_blk[sub_ptr[J]:sub_ptr[J + 1]]) for J in range(nb)}
    owned = {J: [J] for J in range(nb)}
    owner = list(range(nb))       # molecule -> group id

    def candidates(i):
        return {owner[b] for b in rows[i]} - {i}

    while True:
        best = None
        for i in sorted(rows):
            for j in candidates(i):
                if j < i:
                    continue   # symmetric patterns: each pair is seen from its smaller id
                a, b = i, j
                if len(owned[a]) + len(owned[b]) > max_own:
                    continue
                mi, mj = len(rows[a]), len(rows[b])
                mij = len(rows[a] & rows[b])
                mu = mi + mj - mij
                if not mu ** 3 < mi ** 3 + mj ** 3:
                    continue
                key = (min(mj - mij, mi - mij), -(mi ** 3 + mj ** 3 - mu ** 3), a, b)
                if best is None or key < best:
                    best = key
        if best is None:
            break
        _, _, a, b = best
        rows[a] |= rows.pop(b)
        owned[a] = sorted(owned[a] + owned.pop(b))
        for J in owned[a]:
            owner[J] = a
    order = sorted(rows, key=lambda g: owned[g][0])
    grp_ptr, grp_blk, own_ptr, own_J = [0], [], [0], []
    for g in order:
        grp_blk.extend(sorted(rows[g]))
        grp_ptr.append(len(grp_blk))
        own_J.extend(owned[g])
        own_ptr.append(len(own_J))
    return (np.array(grp_ptr, np.int64), np.array(grp_blk, np.int64),
            np.array(own_ptr, np.int64), np.array(own_J, np.int64))


def cubic_cost(ptr):
    """sum over submatrices of m^3 (blocks): the paper's cubic work metric."""
    m = np.diff(np.asarray(ptr, np.int64)).astype(np.float64)
    return float((m ** 3).sum())
