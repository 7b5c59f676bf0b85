"""The seeded generator: determinism, geometry and the structure it promises."""
import numpy as np

import synth
from synth.water import neighbour_pairs, MIN_SEP


def test_deterministic_per_seed():
    a = synth.water_cube(64, 0.6, config_id=1)
    b = synth.water_cube(64, 0.6, config_id=1)
    assert np.array_equal(a.centres, b.centres)
    assert np.array_equal(a.K.val, b.K.val) and np.array_equal(a.S.val, b.S.val)
    c = synth.water_cube(64, 0.6, config_id=7)
    assert not np.array_equal(a.centres, c.centres)


def test_geometry_and_density(box64):
    s = box64
    n = s.nmol
    assert abs(n / np.prod(s.box) - 33.4) < 1e-9
    d = synth.min_image(s.centres[:, None] - s.centres[None], s.box)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(n) * 10
    assert r.min() >= MIN_SEP


def test_matrices_symmetric_spd(box64):
    from oracle.nolsm import dense
    s = box64
    K, S = dense(s.K), dense(s.S)
    assert np.array_equal(K, K.T) and np.array_equal(S, S.T)
    np.linalg.cholesky(S)
    assert np.allclose(np.diag(S), 1.1)
    onsite = np.diag(K).reshape(-1, 6)
    assert np.all((onsite[:, :4] >= -1.1) & (onsite[:, :4] <= -0.9))
    assert np.all((onsite[:, 4:] >= 0.9) & (onsite[:, 4:] <= 1.1))


def test_kdtree_pairs_match_brute_force():
    s = synth.water_cube(2500, 0.9, config_id=9)
    iu, ju = neighbour_pairs(s.centres, s.box, 0.9)   # KD-tree path (n > 2048)
    d = synth.min_image(s.centres[:, None] - s.centres[None], s.box)
    r = np.sqrt((d ** 2).sum(-1))
    bi, bj = np.nonzero(np.triu(r < 0.9, k=1))
    assert np.array_equal(iu, bi) and np.array_equal(ju, bj)


def test_slab_two_densities():
    s = synth.water_slab(config_id=44, r_c=1.2, n_dense=600, n_dilute=600,
                         box=np.array([3.0, 3.0, 6.24]), z_split=600 / 33.4 / 9.0)
    z = s.centres[:, 2]
    split = 600 / 33.4 / 9.0
    assert (z[:600] < split).all() and (z[600:] >= split).all()
    m = np.diff(s.K.row_ptr)
    assert m[:600].mean() > 1.5 * m[600:].mean()
