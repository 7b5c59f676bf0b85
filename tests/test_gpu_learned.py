"""Learned spectral bounds: trained on the GPU by the library's own kernels on
oracle eigensolve labels (tests/golden/mlp_train.npz, written by
oracle/make_training_set.py), then evaluated on a trajectory of the
homogeneous 4096-molecule system against the Gershgorin scale at the same
precision: fewer Newton-Schulz iterations at no worse band-energy error."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import nolsm as o

pytestmark = pytest.mark.gpu
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mlp_train.npz")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    from paper_2104_08245_amd import learned
    d = np.load(DATA)
    say(f"[gpu] training MLP on {len(d['features'])} labelled submatrices")
    return learned.train(d["features"], d["labels"], epochs=60, log=say)


def test_training_reduces_loss(trained):
    h = trained["history"]
    assert h[-1][1] < 0.5 * h[0][1]


def test_predictions_bound_the_spectrum_mostly(trained):
    from paper_2104_08245_amd import learned
    d = np.load(DATA)
    F, lab = d["features"][-2000:], d["labels"][-2000:]
    pred = learned.predict(trained["params"], trained["norm"], F)
    glo, ghi = learned.gershgorin_box(F)
    rho_hat = np.maximum(np.abs(pred[:, 0] * glo), np.abs(pred[:, 1] * ghi))
    rho = np.maximum(np.abs(lab[:, 0]), np.abs(lab[:, 1]))
    rho_g = np.maximum(np.abs(glo), np.abs(ghi))
    # the learned radius is much tighter than Gershgorin's
    assert np.median(rho_hat / rho) < np.median(rho_g / rho)
    # with the 1.05 safety factor, scaled spectra stay inside the NS
    # convergence region (|x| < sqrt 3) everywhere
    assert np.all(rho / (1.05 * rho_hat) < np.sqrt(3))


def test_learned_bounds_save_iterations_on_trajectory(trained):
    import torch
    from paper_2104_08245_amd import Solver, _lib as L
    frames = synth.trajectory(nframes=3)
    res = {}
    for mode in ("gershgorin", "learned"):
        its, fb, dEs = [], 0, []
        for f, s in enumerate(frames):
            kw = {}
            if mode == "learned":
                kw = dict(bounds=L.BOUNDS_LEARNED, d_mlp=trained["params"].data_ptr(),
                          d_mlp_norm=trained["norm"].data_ptr())
            say(f"[gpu] frame {f} {mode}")
            sv = Solver(s, prec="fp16", **kw)
            sv.run()
            torch.cuda.synchronize()
            st = sv.host_stats()
            assert np.all(st["status"] == 0)
            its.append(st["iters"])
            fb += int(st["fallback"].sum())
            for J in (5, 1000, 3000):
                r = o.solve_molecule(s, J)
                dEs.append(abs(st["energy_KD"][J] - r.E_J))
        res[mode] = (np.concatenate(its), fb, np.array(dEs))
        say(f"{mode}: mean iters {res[mode][0].mean():.3f}, fallbacks {fb}, max |dE| {res[mode][2].max():.2e}")
    g, l = res["gershgorin"], res["learned"]
    assert l[0].mean() < g[0].mean()
    assert l[2].max() <= max(2.0 * g[2].max(), 1e-3)


# ------------------------------------------------ the symmetric (bench) path
DATA_SYM = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mlp_train_sym.npz")


@pytest.mark.parametrize("inverse,subst_fp32", [("cholesky", 0), ("cholesky_apply_fp32", 0),
                                                ("cholesky_apply_fp32", 1)])
def test_features_of_symmetric_matrix_match_oracle(box64, inverse, subst_fp32):
    # with sym_sign the features are those of A~ = L^-1 K_J L^-T - mu I
    import torch
    from oracle import mlp
    from paper_2104_08245_amd import Solver, _lib as L
    inv = {"cholesky": L.INV_CHOLESKY, "cholesky_apply_fp32": L.INV_CHOLESKY_APPLY_FP32}[inverse]
    mu = 0.05
    sv = Solver(box64, prec="fp16", device="cuda:0", sym_sign=1, inverse=inv, subst_fp32=subst_fp32)
    sv.want_features()
    sv.run(mu=mu)
    torch.cuda.synchronize()
    f = sv.features.cpu().numpy().reshape(box64.nmol, 12)
    # FP64 application: to the FP32 rounding of the features; FP32
    # application: kappa(L) 2^-24 on A~ itself, on the FP32 matrix cores
    # or (default) as split FP16 products with about 2^-22 per operand
    tol = 1e-5 if inverse == "cholesky" else 1e-4
    for J in range(0, box64.nmol, 3):
        KJ, SJ, idx, p = o.submatrix(box64, J)
        ref = mlp.features_symmetric(KJ, SJ, mu)
        assert np.allclose(f[J], ref, rtol=tol, atol=tol), (J, f[J], ref)


@pytest.fixture(scope="module")
def trained_sym():
    import torch
    assert torch.cuda.is_available()
    from paper_2104_08245_amd import learned
    d = np.load(DATA_SYM)
    say(f"[gpu] training MLP on the symmetric-matrix features of {len(d['features'])} submatrices")
    return learned.train(d["features"], d["labels"], epochs=60, log=say)


def test_learned_bounds_on_symmetric_path_save_iterations(trained_sym):
    # the benchmarked path: symmetric iteration, FP64 factor applied in FP32
    import torch
    from paper_2104_08245_amd import Solver, _lib as L
    frames = synth.trajectory(nframes=2)
    res = {}
    for mode in ("gershgorin", "learned"):
        its, fb, dEs = [], 0, []
        for f, s in enumerate(frames):
            kw = dict(sym_sign=1, inverse=L.INV_CHOLESKY_APPLY_FP32)
            if mode == "learned":
                kw.update(bounds=L.BOUNDS_LEARNED, d_mlp=trained_sym["params"].data_ptr(),
                          d_mlp_norm=trained_sym["norm"].data_ptr())
            say(f"[gpu] symmetric frame {f} {mode}")
            sv = Solver(s, prec="fp16", **kw)
            sv.run()
            torch.cuda.synchronize()
            st = sv.host_stats()
            assert np.all(st["status"] == 0)
            its.append(st["iters"])
            fb += int(st["fallback"].sum())
            for J in (5, 1000, 3000):
                r = o.solve_molecule(s, J)
                dEs.append(abs(st["energy_KD"][J] - r.E_J))
        res[mode] = (np.concatenate(its), fb, np.array(dEs))
        say(f"symmetric {mode}: mean iters {res[mode][0].mean():.3f}, fallbacks {fb}, "
            f"max |dE| {res[mode][2].max():.2e}")
    g, l = res["gershgorin"], res["learned"]
    assert l[0].mean() < g[0].mean()
    assert l[2].max() <= max(2.0 * g[2].max(), 1e-3)
