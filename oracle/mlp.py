"""FP64 CPU oracle of the learned spectral-bound model.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

The paper fixes the scaling only qualitatively: the matrix is rescaled before
the sign iteration so that the iteration converges (Sec. III-B.2, after
Eq. NS2). The learned part predicts the extreme eigenvalues of A_J from cheap
O(n^2) features, so that the scale can be tighter than a Gershgorin bound.

Model: 12 features -> Linear(12,64) -> SiLU -> Linear(64,64) -> SiLU ->
Linear(64,2). Targets are the normalised extremes (lambda_min / G_lo,
lambda_max / G_hi) where [G_lo, G_hi] is the intersection of the row and
column Gershgorin intervals. Loss: mean over batch and both outputs of
w * (pred - y)^2 with w = 4 where the prediction underestimates (pred < y),
else 1. Optimiser: Adam (Kingma & Ba) with bias correction.

Parameter packing (float, 5122 values): W1[64][12], b1[64], W2[64][64],
b2[64], W3[2][64], b3[2]; W row-major as [out][in].
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

NF = 12
H = 64
NO = 2
SIZES = [(H, NF), (H,), (H, H), (H,), (NO, H), (NO,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)
UNDER_WEIGHT = 4.0


def unpack(theta):
    out, o = [], 0
    for s in SIZES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def init_params(rng):
    """He-style uniform init, biases zero."""
    theta = np.zeros(NPARAM)
    parts = unpack(theta)
    for W in (parts[0], parts[2], parts[4]):
        fan_in = W.shape[1]
        W[...] = rng.uniform(-1, 1, W.shape) * np.sqrt(3.0 / fan_in)
    return theta


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    out = h2 @ W3.T + b3
    return out, (x, z1, h1, z2, h2)


def loss(out, y):
    d = out - y
    w = np.where(d < 0, UNDER_WEIGHT, 1.0)
    return float((w * d * d).mean())


def loss_and_grad(theta, x, y):
    """Loss and its exact gradient by hand-written backpropagation."""
    out, (x, z1, h1, z2, h2) = forward(theta, x)
    B = x.shape[0]
    d = out - y
    w = np.where(d < 0, UNDER_WEIGHT, 1.0)
    L = float((w * d * d).mean())
    g_out = 2.0 * w * d / (B * NO)
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    grad = np.zeros_like(theta)
    gW1, gb1, gW2, gb2, gW3, gb3 = unpack(grad)
    gW3[...] = g_out.T @ h2
    gb3[...] = g_out.sum(0)
    g_h2 = g_out @ W3
    g_z2 = g_h2 * dsilu(z2)
    gW2[...] = g_z2.T @ h1
    gb2[...] = g_z2.sum(0)
    g_h1 = g_z2 @ W2
    g_z1 = g_h1 * dsilu(z1)
    gW1[...] = g_z1.T @ x
    gb1[...] = g_z1.sum(0)
    return L, grad


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# Features and labels of one A_J = S_J^-1 K_J - mu I
# --------------------------------------------------------------------------

FEATURE_NAMES = ["log_n", "diag_mean", "diag_std", "diag_min", "diag_max",
                 "row_radius_mean", "row_radius_max", "row_glo", "row_ghi",
                 "col_glo", "col_ghi", "frob_over_sqrt_n"]


def features(A):
    n = A.shape[0]
    d = np.diag(A)
    off = np.abs(A) - np.diag(np.abs(d))
    rr = off.sum(axis=1)
    cr = off.sum(axis=0)
    return np.array([np.log(n), d.mean(), d.std(), d.min(), d.max(), rr.mean(), rr.max(),
                     (d - rr).min(), (d + rr).max(), (d - cr).min(), (d + cr).max(),
                     np.linalg.norm(A) / np.sqrt(n)])


def symmetric_similar(KJ, SJ, mu):
    """A~ = L^-1 K_J L^-T - mu I with S_J = L L^T (lower Cholesky factor):
    similar to A_J = S_J^-1 K_J - mu I (A_J = L^-T A~ L^T), so the same
    spectrum, and symmetric. The symmetric sign iteration runs on it; its
    features are those of this matrix."""
    L = sla.cholesky(SJ, lower=True)
    W = sla.solve_triangular(L, KJ, lower=True)            # L^-1 K
    At = sla.solve_triangular(L, W.T, lower=True).T       # (L^-1 (L^-1 K)^T)^T = L^-1 K L^-T
    return At - mu * np.eye(KJ.shape[0])


def features_symmetric(KJ, SJ, mu):
    """The 12 features of A~ (symmetric_similar)."""
    return features(symmetric_similar(KJ, SJ, mu))


def gershgorin_box(f):
    """Intersection of the row and column Gershgorin intervals from a feature
    vector: (G_lo, G_hi)."""
    return max(f[7], f[9]), min(f[8], f[10])


def labels(KJ, SJ, mu):
    """Extreme eigenvalues of A_J = S_J^-1 K_J - mu I, from the symmetric-definite
    generalized eigenproblem (K_J - mu S_J) v = lambda S_J v."""
    n = KJ.shape[0]
    lo = sla.eigh(KJ - mu * SJ, SJ, eigvals_only=True, subset_by_index=[0, 0])[0]
    hi = sla.eigh(KJ - mu * SJ, SJ, eigvals_only=True, subset_by_index=[n - 1, n - 1])[0]
    return float(lo), float(hi)


def targets(f, lam_lo, lam_hi):
    glo, ghi = gershgorin_box(f)
    return np.array([lam_lo / glo, lam_hi / ghi])


def scale_from_prediction(f, pred, safety=1.05):
    """Scale c_J = 1 / (safety * rho_hat), never below the Gershgorin scale."""
    glo, ghi = gershgorin_box(f)
    rho_g = max(abs(glo), abs(ghi))
    rho_hat = max(abs(pred[0] * glo), abs(pred[1] * ghi))
    c = 1.0 / (safety * rho_hat) if rho_hat > 0 else 1.0 / rho_g
    return max(c, 1.0 / rho_g)
