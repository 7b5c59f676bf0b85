"""Pins of the MLP oracle: hand-written backpropagation against central finite
differences, Adam against its closed-form first step, features against their
definitions on a matrix with a known answer, labels against a dense eigensolve."""
import numpy as np
import scipy.linalg as sla

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(rng)
    x = rng.standard_normal((7, mlp.NF))
    y = rng.uniform(0.2, 1.0, (7, mlp.NO))
    L, g = mlp.loss_and_grad(theta, x, y)
    assert abs(L - mlp.loss(mlp.forward(theta, x)[0], y)) < 1e-15
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, 300, replace=False)
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(mlp.forward(tp, x)[0], y) - mlp.loss(mlp.forward(tm, x)[0], y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9


def test_adam_first_step_is_signed_lr():
    # with zero moments, the bias-corrected first step is lr * g / (|g| + eps')
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 3.0, -0.25])
    t2, m, v = mlp.adam_step(theta, g, np.zeros(5), np.zeros(5), 1, lr=1e-3, eps=0.0)
    assert np.allclose(t2, -1e-3 * np.sign(g), rtol=0, atol=1e-15)


def test_features_of_known_matrix():
    A = np.array([[2.0, -1.0, 0.0], [0.5, -3.0, 1.0], [0.0, 2.0, 1.0]])
    f = mlp.features(A)
    assert np.isclose(f[0], np.log(3))
    assert np.isclose(f[1], 0.0) and np.isclose(f[3], -3.0) and np.isclose(f[4], 2.0)
    # row radii 1, 1.5, 2; column radii 0.5, 3, 1
    assert np.isclose(f[5], 1.5) and np.isclose(f[6], 2.0)
    assert np.isclose(f[7], -4.5) and np.isclose(f[8], 3.0)
    assert np.isclose(f[9], -6.0) and np.isclose(f[10], 2.5)
    assert np.isclose(f[11], np.sqrt((A ** 2).sum() / 3))


def test_labels_are_extreme_generalized_eigenvalues():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((20, 20))
    S = M @ M.T + 20 * np.eye(20)
    K = rng.standard_normal((20, 20)); K = K + K.T
    lo, hi = mlp.labels(K, S, 0.3)
    w = np.linalg.eigvals(np.linalg.solve(S, K) - 0.3 * np.eye(20)).real
    assert np.isclose(lo, w.min()) and np.isclose(hi, w.max())


def test_scale_never_below_gershgorin():
    f = np.zeros(12); f[7], f[8], f[9], f[10] = -3.0, 2.0, -2.5, 2.5
    # prediction claims a spectrum 10x larger than Gershgorin: clamp to 1/rho_G
    assert mlp.scale_from_prediction(f, np.array([10.0, 10.0])) == 1.0 / 2.5
    c = mlp.scale_from_prediction(f, np.array([0.5, 0.5]))
    assert np.isclose(c, 1.0 / (1.05 * 1.25))


def test_symmetric_similar_matrix_and_its_features():
    # A~ = L^-1 K L^-T - mu I on a submatrix of the 64-molecule box: symmetric,
    # with the spectrum of A_J (the generalized eigenvalues of (K - mu S, S)),
    # enclosed by its Gershgorin box; its row and column radii coincide, and
    # a planted transposition (L^-T K L^-1) breaks the spectrum check
    import synth
    from oracle import nolsm as o
    s = synth.make_config(1)
    mu = 0.1
    for J in (0, 17, 63):
        KJ, SJ, idx, p = o.submatrix(s, J)
        At = mlp.symmetric_similar(KJ, SJ, mu)
        ref = sla.eigh(KJ - mu * SJ, SJ, eigvals_only=True)
        assert np.abs(At - At.T).max() <= 1e-12 * np.abs(At).max()
        ev = np.linalg.eigvalsh((At + At.T) / 2)
        assert np.abs(ev - ref).max() <= 1e-10 * np.abs(ref).max()
        f = mlp.features_symmetric(KJ, SJ, mu)
        assert np.allclose(f[7:9], f[9:11], rtol=1e-12, atol=1e-12)
        glo, ghi = mlp.gershgorin_box(f)
        assert glo <= ref.min() + 1e-12 and ref.max() <= ghi + 1e-12
        assert abs(f[1] - np.trace(At) / At.shape[0]) <= 1e-12 * np.abs(At).max()
        L = sla.cholesky(SJ, lower=True)
        wrong = sla.solve_triangular(L.T, sla.solve_triangular(L.T, KJ, lower=False).T, lower=False)
        assert np.abs(np.linalg.eigvalsh((wrong + wrong.T) / 2) - mu - ref).max() > 1e-6
