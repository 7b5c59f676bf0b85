"""Pins of the oracle's energy-weighted density matrix T_J(W) = T_J(D) T_J(K)
T_J(D) (Sec. III-B.2, written back column by column like D) against facts
that do not come from the oracle itself.

W1 full-cell closed form: when the cutoff covers the whole periodic cell every
   submatrix is the full matrix, so W must equal C_occ diag(eps_occ) C_occ^T
   of the generalized eigenproblem K c = eps S c (c^T S c = 1), and
   Tr(W S) = sum of the occupied eps.
W2 block-diagonal case: per block, the same closed form.
W3 per submatrix, for a converged sign: T_J(D) = P S_J^-1 with P = (I - X)/2 a
   projector that commutes with A_J = S_J^-1 K_J - mu I, so the owned columns
   equal (A_J + mu I) Dcols_J.
Mutation checks plant plausible mistakes in the W step and show that W1
rejects each of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import nolsm as o


def full_cell(nmol, r_c, cid):
    s = synth.water_cube(nmol, r_c, config_id=cid)
    assert r_c > s.box[0] * np.sqrt(3) / 2, "cutoff must cover the whole cell"
    return s


def exact_W(Kd, Sd, mu):
    w, C = sla.eigh(Kd, Sd)
    occ = w < mu
    Co = C[:, occ]
    return (Co * w[occ]) @ Co.T, w, occ


def assembled_W(s, r):
    return o.dense_from_pattern(s.K.nb, s.K.bs, r.plan["D_row_ptr"], r.plan["D_col_idx"], r.W_val)


@pytest.mark.parametrize("nmol,r_c,cid,mu", [(8, 0.6, 101, 0.0), (16, 0.7, 102, 0.0),
                                              (8, 0.6, 103, 1.1), (8, 0.6, 104, -0.5)])
def test_w1_full_cell_equals_closed_form(nmol, r_c, cid, mu):
    s = full_cell(nmol, r_c, cid)
    r = o.nolsm(s, mu=mu, want_w=True)
    assert np.all(r.status == o.OK)
    Kd, Sd = o.dense(s.K), o.dense(s.S)
    Wex, w, occ = exact_W(Kd, Sd, mu)
    W = assembled_W(s, r)
    assert np.linalg.norm(W - Wex) / np.linalg.norm(Wex) <= 1e-10
    assert abs(np.trace(W @ Sd) - w[occ].sum()) < 1e-9 * max(1.0, abs(w[occ].sum()))


def test_w2_block_diagonal():
    s = synth.water_cube(64, 0.2, config_id=105)
    assert s.K.nnzb == 64
    r = o.nolsm(s, want_w=True)
    for J in range(64):
        WJ, w, occ = exact_W(s.K.val[J], s.S.val[J], 0.0)
        assert np.allclose(r.Wcols[J], WJ, rtol=0, atol=1e-12 * np.abs(WJ).max())


def test_w3_projector_identity(box64):
    s = box64
    for J in (0, 17, 40, 63):
        r = o.solve_molecule(s, J, want_w=True)
        assert r.status == o.OK
        n = r.A.shape[0]
        ref = (r.A + s.mu * np.eye(n)) @ r.Dcols
        assert np.linalg.norm(r.Wcols - ref) <= 1e-9 * np.linalg.norm(ref)


_ORIG = o.solve_submatrix


def _mutant(kind):
    def solve(KJ, SJ, p, bs, mu, tol=1e-10, max_iter=100, scale=None, want_w=False):
        r = _ORIG(KJ, SJ, p, bs, mu, tol, max_iter, scale, want_w)
        if r.Dcols is None or not want_w:
            return r
        n = KJ.shape[0]
        DJ = 0.5 * (np.eye(n) - r.X) @ np.linalg.inv(SJ)
        cols = slice(p * bs, (p + 1) * bs)
        if kind == "one_D":          # W = D K instead of D K D
            r.Wcols = (DJ @ KJ)[:, cols]
        elif kind == "S_for_K":      # overlap in place of the Hamiltonian
            r.Wcols = DJ @ SJ @ r.Dcols
        elif kind == "no_projector":  # S^-1 K S^-1 without the projector
            Sinv = np.linalg.inv(SJ)
            r.Wcols = (Sinv @ KJ @ Sinv)[:, cols]
        elif kind == "sign_flip":    # (I + X)/2: the unoccupied projector
            Du = 0.5 * (np.eye(n) + r.X) @ np.linalg.inv(SJ)
            r.Wcols = Du @ KJ @ Du[:, cols]
        return r
    return solve


@pytest.mark.parametrize("kind", ["one_D", "S_for_K", "no_projector", "sign_flip"])
def test_w_pins_reject_planted_mistakes(kind, monkeypatch):
    s = full_cell(8, 0.6, 103)
    mu = 1.1
    Wex, _, _ = exact_W(o.dense(s.K), o.dense(s.S), mu)
    monkeypatch.setattr(o, "solve_submatrix", _mutant(kind))
    r = o.nolsm(s, mu=mu, want_w=True)
    W = assembled_W(s, r)
    assert np.linalg.norm(W - Wex) / np.linalg.norm(Wex) > 1e-6
