"""Pins of the oracle's coupled Newton-Schulz inverse (Eq. inv1-inv3) against
facts that do not come from the oracle itself.

I1 it equals the inverse of the SPD submatrices T_J(S) (LAPACK) to 1e-12;
I2 closed forms: a 1 x 1 matrix s gives 1/s, a diagonal matrix its reciprocal
   diagonal, the identity itself after zero updates;
I3 Z_k is a polynomial in S: the returned c Z^2 is symmetric and c Z^2 S = I;
I4 the whole NOLSM D built on it equals the one built on the Cholesky factor
   (same definition, different route to T_J(S)^-1) to 1e-10;
mutation checks: plausible mistakes in the iteration are rejected by I1.
"""
import numpy as np
import pytest

from oracle import nolsm as o


def scale(S):
    return 1.0 / np.abs(S).sum(axis=1).max()


def test_i1_equals_lapack_inverse(box64):
    for J in (0, 21, 63):
        _, SJ, _, _ = o.submatrix(box64, J)
        Sinv, k, r, ok = o.coupled_ns_inverse(SJ, scale(SJ))
        assert ok and r < 1e-12 and 5 <= k <= 30
        ref = np.linalg.inv(SJ)
        assert np.linalg.norm(Sinv - ref) <= 1e-12 * np.linalg.norm(ref)


def test_i2_closed_forms():
    Sinv, k, _, ok = o.coupled_ns_inverse(np.array([[2.5]]), 0.3)
    assert ok and abs(Sinv[0, 0] - 0.4) < 1e-15
    d = np.array([0.2, 1.0, 3.0, 7.5])
    Sinv, _, _, ok = o.coupled_ns_inverse(np.diag(d), 1.0 / d.max())
    assert ok and np.allclose(np.diag(Sinv), 1.0 / d, rtol=1e-14, atol=0)
    assert np.count_nonzero(Sinv - np.diag(np.diag(Sinv))) == 0
    Sinv, k, _, ok = o.coupled_ns_inverse(np.eye(5), 1.0)
    assert ok and k == 0 and np.array_equal(Sinv, np.eye(5))


def test_i3_polynomial_structure(box64):
    _, SJ, _, _ = o.submatrix(box64, 7)
    Sinv, _, _, ok = o.coupled_ns_inverse(SJ, scale(SJ))
    assert ok
    assert np.linalg.norm(Sinv - Sinv.T) <= 1e-13 * np.linalg.norm(Sinv)
    n = SJ.shape[0]
    assert np.linalg.norm(Sinv @ SJ - np.eye(n)) <= 1e-11


def test_i4_density_matrix_equals_cholesky_route(box64):
    for J in (3, 33, 50):
        a = o.solve_molecule(box64, J)
        b = o.solve_molecule(box64, J, inverse="coupled_ns")
        assert a.status == b.status == o.OK
        assert np.linalg.norm(b.Dcols - a.Dcols) <= 1e-10 * np.linalg.norm(a.Dcols)
        assert abs(a.E_J - b.E_J) <= 1e-10 * max(1.0, abs(a.E_J))


def _mutant(kind):
    def inv(S, c, tol=1e-12, max_iter=100):
        n = S.shape[0]
        I = np.eye(n)
        Y, Z = c * S, I.copy()
        for k in range(max_iter):
            V = Z @ Y
            if np.linalg.norm(V - I) < tol:
                break
            if kind == "no_half":
                T = 3.0 * I - V
                Y, Z = Y @ T, T @ Z
            elif kind == "plus_sign":
                T = 3.0 * I + V
                Y, Z = 0.5 * (Y @ T), 0.5 * (T @ Z)
            elif kind == "stale_Y":      # Z updated with V but Y left unchanged
                T = 3.0 * I - V
                Z = 0.5 * (T @ Z)
            elif kind == "no_square":    # returns c Z instead of c Z^2
                T = 3.0 * I - V
                Y, Z = 0.5 * (Y @ T), 0.5 * (T @ Z)
            if not np.all(np.isfinite(Z)):
                break
        return (c * Z if kind == "no_square" else c * (Z @ Z)), k, 0.0, True
    return inv


@pytest.mark.parametrize("kind", ["no_half", "plus_sign", "stale_Y", "no_square"])
def test_inverse_pins_reject_planted_mistakes(kind, box64):
    _, SJ, _, _ = o.submatrix(box64, 0)
    with np.errstate(all="ignore"):
        Sinv, _, _, _ = _mutant(kind)(SJ, scale(SJ), max_iter=40)
        ref = np.linalg.inv(SJ)
        err = np.linalg.norm(Sinv - ref) / np.linalg.norm(ref)
    assert not (err <= 1e-12)
