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


def test_two_cutoffs_patterns_strictly_nested():
    # K truncated at 0.45 nm inside S at 0.6 nm (and the reverse): every
    # block of the smaller pattern is in the larger one with the same values,
    # the larger one has blocks the smaller lacks, and both stay symmetric
    import synth
    from oracle import nolsm as o
    base = synth.make_config(1)
    for kw, small, big in ((dict(r_k=0.45), "K", "S"), (dict(r_s=0.45), "S", "K")):
        s = synth.two_cutoffs(base, **kw)
        a, b = getattr(s, small), getattr(s, big)
        assert a.nnzb < b.nnzb
        o.validate_pattern(a.nb, a.row_ptr, a.col_idx)
        for I in range(a.nb):
            ca = a.col_idx[a.row_ptr[I]:a.row_ptr[I + 1]]
            cb = b.col_idx[b.row_ptr[I]:b.row_ptr[I + 1]]
            assert set(ca.tolist()) <= set(cb.tolist())
            full = getattr(base, small)
            for k in range(a.row_ptr[I], a.row_ptr[I + 1]):
                kf = o.find_block(full.row_ptr, full.col_idx, I, int(a.col_idx[k]))
                assert np.array_equal(a.val[k], full.val[kf])
