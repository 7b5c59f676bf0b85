"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, never against a second copy of itself.

P1 full-cell closed form: when the cutoff covers the whole periodic cell every
   submatrix is the full matrix, so NOLSM must equal the exact density matrix
   C_occ C_occ^T of the generalized eigenproblem K c = eps S c (Eq. purification),
   with Tr(DS) = #occupied and E = sum of occupied eps (Eq. e_elec).
P2 block-diagonal case: a cutoff below the minimum separation leaves N(J) = {J}.
P3 per-submatrix invariants: X^2 = I, S_J-idempotency of D_J, Tr(S_J D_J) =
   number of negative generalized eigenvalues, S_J X symmetric.
P4 textbook special cases: S = I, mu outside the spectrum, a 1x1 problem.
P5 Gershgorin enclosure of the spectrum of A_J.
P6 indexing: N(J) equals a brute-force distance search; D keeps the merged
   pattern (Sec. III-B.2: same sparsity as the input).
Mutation checks plant plausible mistakes in a copy of the oracle's
per-submatrix step and show that the pins reject each of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import nolsm as o


def full_cell(nmol, r_c, cid):
    s = synth.water_cube(nmol, r_c, config_id=cid)
    L = s.box[0]
    assert r_c > L * np.sqrt(3) / 2, "cutoff must cover the whole cell"
    assert s.K.nnzb == nmol * nmol
    return s


def exact_D(Kd, Sd, mu):
    w, C = sla.eigh(Kd, Sd)
    occ = w < mu
    Co = C[:, occ]
    return Co @ Co.T, w, occ


def assembled(s, r):
    return o.dense_from_pattern(s.K.nb, s.K.bs, r.plan["D_row_ptr"], r.plan["D_col_idx"], r.D_val)


@pytest.mark.parametrize("nmol,r_c,cid,mu", [(8, 0.6, 101, 0.0), (16, 0.7, 102, 0.0),
                                              (8, 0.6, 103, 1.1), (8, 0.6, 104, -0.5)])
def test_p1_full_cell_equals_eigendecomposition(nmol, r_c, cid, mu):
    s = full_cell(nmol, r_c, cid)
    r = o.nolsm(s, mu=mu)
    assert np.all(r.status == o.OK)
    Kd, Sd = o.dense(s.K), o.dense(s.S)
    Dex, w, occ = exact_D(Kd, Sd, mu)
    D = assembled(s, r)
    assert np.linalg.norm(D - Dex) / np.linalg.norm(Dex) <= 1e-10
    assert abs(np.trace(D @ Sd) - occ.sum()) < 1e-9
    assert abs(r.N.sum() - occ.sum()) < 1e-9
    assert abs(r.E.sum() - w[occ].sum()) < 1e-9 * max(1.0, abs(w[occ].sum()))
    if mu == 0.0:
        assert occ.sum() == 4 * nmol


def test_p2_block_diagonal():
    s = synth.water_cube(64, 0.2, config_id=105)
    assert s.K.nnzb == 64
    r = o.nolsm(s)
    for J in range(64):
        KJ = s.K.val[J]
        SJ = s.S.val[J]
        DJ, w, occ = exact_D(KJ, SJ, 0.0)
        assert np.allclose(r.Dcols[J], DJ, rtol=0, atol=1e-12 * np.abs(DJ).max())
        assert occ.sum() == 4
        assert abs(r.N[J] - 4) < 1e-10


def test_p3_per_submatrix_invariants(box64):
    s = box64
    r = o.nolsm(s, molecules=range(0, 64, 7), keep_x=True)
    for J in range(0, 64, 7):
        KJ, SJ, idx, p = o.submatrix(s, J)
        X, A = r.xs[J]
        n = KJ.shape[0]
        assert np.linalg.norm(X @ X - np.eye(n)) < 1e-10
        Sinv = np.linalg.inv(SJ)
        DJ = 0.5 * (np.eye(n) - X) @ Sinv
        assert np.linalg.norm(DJ @ SJ @ DJ - DJ) <= 1e-9 * np.linalg.norm(DJ)
        nu = int((sla.eigh(KJ, SJ, eigvals_only=True) < 0).sum())
        assert abs(np.trace(SJ @ DJ) - nu) < 1e-8
        SX = SJ @ X
        assert np.linalg.norm(SX - SX.T) < 1e-9 * np.linalg.norm(SX)
        assert np.linalg.norm(X @ A - A @ X) < 1e-9 * np.linalg.norm(A)
        # the written-back columns are exactly D_J's owned columns
        assert np.allclose(r.Dcols[J], DJ[:, 6 * p:6 * p + 6], atol=1e-12, rtol=0)


def test_p4_identity_overlap_is_eigenprojector():
    s = full_cell(8, 0.6, 106)
    eye_blocks = np.zeros_like(s.S.val)
    for I in range(s.S.nb):
        k = o.find_block(s.S.row_ptr, s.S.col_idx, I, I)
        eye_blocks[k] = np.eye(6)
    s.S.val = eye_blocks
    r = o.nolsm(s)
    w, V = np.linalg.eigh(o.dense(s.K))
    P = V[:, w < 0] @ V[:, w < 0].T
    D = assembled(s, r)
    assert np.linalg.norm(D - P) <= 1e-10 * np.linalg.norm(P)


def test_p4_mu_outside_spectrum(box64):
    s = box64
    Js = [0, 17, 40]
    hi = o.nolsm(s, mu=50.0, molecules=Js)
    lo = o.nolsm(s, mu=-50.0, molecules=Js)
    for J in Js:
        KJ, SJ, idx, p = o.submatrix(s, J)
        Sinv = np.linalg.inv(SJ)
        assert np.allclose(hi.Dcols[J], Sinv[:, 6 * p:6 * p + 6], atol=1e-10, rtol=0)
        assert np.abs(lo.Dcols[J]).max() < 1e-12
        assert abs(hi.N[J] - 6) < 1e-10 and abs(lo.N[J]) < 1e-10


@pytest.mark.parametrize("k,sv,mu", [(0.3, 2.0, 0.5), (0.3, 2.0, 0.1), (-1.0, 0.5, 0.0)])
def test_p4_scalar(k, sv, mu):
    K = synth.BlockCSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32),
                       np.array([[[k]]]))
    S = synth.BlockCSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32),
                       np.array([[[sv]]]))
    sysm = synth.System(np.ones(3), 1.0, np.zeros((1, 3)), np.zeros((1, 1, 3)),
                        np.zeros((1, 1)), K, S, mu=mu)
    r = o.nolsm(sysm)
    expect = (1.0 if k / sv < mu else 0.0) / sv
    assert abs(r.D_val[0, 0, 0] - expect) < 1e-14


def test_p5_gershgorin_encloses_spectrum(box64):
    s = box64
    for J in (3, 33, 63):
        KJ, SJ, idx, p = o.submatrix(s, J)
        A = np.linalg.solve(SJ, KJ)
        lam = sla.eigh(KJ, SJ, eigvals_only=True)
        (rlo, rhi), (clo, chi) = o.gershgorin(A)
        assert rlo <= lam.min() and lam.max() <= rhi
        assert clo <= lam.min() and lam.max() <= chi
        # the oracle's scale 1/||A||_inf makes every eigenvalue of X_0 lie in [-1, 1]
        assert np.abs(lam).max() * (1.0 / np.abs(A).sum(axis=1).max()) <= 1.0


def test_p6_indexing_brute_force(box64):
    s = box64
    lists, self_pos = o.merge(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    d = synth.min_image(s.centres[:, None] - s.centres[None], s.box)
    r = np.sqrt((d ** 2).sum(-1))
    for J in range(s.nmol):
        brute = np.nonzero(r[:, J] < s.r_c)[0]
        assert np.array_equal(lists[J], brute)
        assert lists[J][self_pos[J]] == J
    plan = o.plan_arrays(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    # D keeps exactly the merged pattern (here K's = S's pattern)
    assert np.array_equal(plan["D_row_ptr"], s.K.row_ptr)
    assert np.array_equal(plan["D_col_idx"], s.K.col_idx)


def test_merge_is_union_of_different_patterns():
    # K tridiagonal, S diagonal + (0,3)/(3,0): N(J) must be the union
    nb = 4
    Kp = {(i, j) for i in range(nb) for j in range(nb) if abs(i - j) <= 1}
    Sp = {(i, i) for i in range(nb)} | {(0, 3), (3, 0)}
    def csr(p):
        rows = [sorted(j for (i, j) in p if i == r) for r in range(nb)]
        rp = np.cumsum([0] + [len(x) for x in rows])
        return rp, np.array([c for x in rows for c in x])
    krp, kci = csr(Kp)
    srp, sci = csr(Sp)
    lists, sp = o.merge(nb, krp, kci, srp, sci)
    assert [l.tolist() for l in lists] == [[0, 1, 3], [0, 1, 2], [1, 2, 3], [0, 2, 3]]
    assert sp.tolist() == [0, 1, 1, 2]


def test_sign_is_scale_invariant(box64):
    s = box64
    KJ, SJ, idx, p = o.submatrix(s, 11)
    a = o.solve_submatrix(KJ, SJ, p, 6, 0.0)
    A = a.A
    (rlo, rhi), (clo, chi) = o.gershgorin(A)
    c2 = 1.0 / min(np.abs(A).sum(axis=1).max(), np.abs(A).sum(axis=0).max())
    b = o.solve_submatrix(KJ, SJ, p, 6, 0.0, scale=c2)
    assert np.linalg.norm(a.Dcols - b.Dcols) <= 1e-10 * np.linalg.norm(a.Dcols)


def test_validate_rejects_bad_patterns():
    rp = np.array([0, 2, 4]); ci = np.array([0, 1, 0, 1])
    o.validate_pattern(2, rp, ci)
    with pytest.raises(o.PatternError):
        o.validate_pattern(2, rp, np.array([1, 0, 0, 1]))       # unsorted
    with pytest.raises(o.PatternError):
        o.validate_pattern(2, np.array([0, 1, 3]), np.array([1, 0, 1]))  # no diag in row 0
    with pytest.raises(o.PatternError):
        o.validate_pattern(2, np.array([0, 2, 3]), np.array([0, 1, 1]))  # asymmetric
    with pytest.raises(o.PatternError):
        o.validate_pattern(2, np.array([0, 2, 4]), np.array([0, 2, 0, 1]))  # out of range


def test_not_spd_and_noconv_flags(box64):
    s = box64
    KJ, SJ, idx, p = o.submatrix(s, 5)
    bad = SJ.copy()
    bad[0, 0] = -1.0
    assert o.solve_submatrix(KJ, bad, p, 6, 0.0).status == o.NOT_SPD
    assert o.solve_submatrix(KJ, SJ, p, 6, 0.0, max_iter=2).status == o.NOCONV


# --------------------------------------------------------------------------
# Mutation checks: each plausible mistake must fail the full-cell pin.
# --------------------------------------------------------------------------

def _mutant(kind):
    def solve(KJ, SJ, p, bs, mu, tol=1e-10, max_iter=100, scale=None, want_w=False):
        n = KJ.shape[0]
        Sinv = np.linalg.inv(SJ)
        A = Sinv @ KJ - (0.0 if kind == "drop_mu" else mu) * np.eye(n)
        if kind == "transpose_A":
            A = KJ @ Sinv - mu * np.eye(n)
        pp = (p + 1) % (n // bs) if kind == "wrong_self" else p
        E = np.zeros((n, bs)); E[pp * bs:(pp + 1) * bs] = np.eye(bs)
        c = 1.0 / np.abs(A).sum(axis=1).max()
        X, it, r, conv = o.newton_schulz_sign(A, c, tol, max_iter)
        if kind == "sign_flip":
            X = -X
        if kind == "left_inverse":
            Dc = 0.5 * Sinv @ ((np.eye(n) - X) @ E)
        else:
            Dc = 0.5 * (Sinv @ E - X @ (Sinv @ E))
        rows = slice(p * bs, (p + 1) * bs)
        return o.SubResult(o.OK, Dc, X, A, it, r, c, float(np.trace(SJ[rows] @ Dc)),
                           float(np.trace(KJ[rows] @ Dc)))
    return solve


@pytest.mark.parametrize("kind", ["drop_mu", "transpose_A", "wrong_self", "sign_flip",
                                  "left_inverse"])
def test_pins_reject_planted_mistakes(kind, monkeypatch):
    s = full_cell(8, 0.6, 103)
    mu = 1.1
    Dex, w, occ = exact_D(o.dense(s.K), o.dense(s.S), mu)
    monkeypatch.setattr(o, "solve_submatrix", _mutant(kind))
    r = o.nolsm(s, mu=mu)
    D = assembled(s, r)
    assert np.linalg.norm(D - Dex) / np.linalg.norm(Dex) > 1e-6


def test_vectorized_gather_equals_plain_gather(box64):
    s = box64
    lists, _ = o.neighbour_lists(s)
    for J in (0, 9, 63):
        a = o.gather(lists[J], 6, s.K.row_ptr, s.K.col_idx, s.K.val)
        b = o.gather_vectorized(lists[J], 6, s.K.row_ptr, s.K.col_idx, s.K.val)
        assert np.array_equal(a, b)


def test_forced_restart_reaches_the_same_sign(box64):
    # the divergence guard's restart (X_{k+1} = c A instead of the update,
    # injected at k = 2) delays the iteration but converges to the same sign
    J = 9
    a = o.solve_molecule(box64, J)
    b = o.solve_molecule(box64, J, restart_at=2)
    assert a.status == b.status == 0
    assert b.iters == a.iters + 3
    assert np.linalg.norm(a.Dcols - b.Dcols) <= 1e-12 * np.linalg.norm(a.Dcols)
