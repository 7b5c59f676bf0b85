"""Degenerate and extreme submatrix sizes, through the C ABI.

- Isolated molecules (cutoff below the closest approach): every N(J) is {J},
  a 6 x 6 submatrix padded to one 64-row tile. The method then reduces to
  the exact density matrix of each molecule on its own (the block-diagonal
  case pinned on the CPU), and the GPU matches the oracle.
- The largest submatrix the library accepts (NOLSM_MAX_ROWS): a full cell of
  501 molecules, where every submatrix is the whole 3006 x 3006 matrix. NOLSM
  is then exact, so every molecule's column block is held to the column
  block of the generalized eigendecomposition's density matrix
  C_occ C_occ^T (LAPACK), in FP64 to 1e-10 and in the mixed precisions to
  their bounds, with the energies E_J = tr(K[cJ, :] D[:, cJ]).
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import nolsm as o

pytestmark = pytest.mark.gpu

MIXED = {"fp16": dict(dcols=5e-3, energy=1e-3), "bf16": dict(dcols=4e-2, energy=1e-2)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def solve(system, prec, **kw):
    from paper_2104_08245_amd import Solver
    import torch
    say(f"[gpu] solve prec={prec} nmol={system.nmol} {kw}")
    sv = Solver(system, prec=prec, device="cuda:0", **kw)
    sv.run()
    torch.cuda.synchronize()
    return sv


@pytest.fixture(scope="module")
def isolated():
    s = synth.water_cube(32, 0.1, config_id=110)
    assert s.K.nnzb == s.nmol   # diagonal blocks only
    return s


@pytest.fixture(scope="module")
def isolated_ref(isolated):
    return o.nolsm(isolated)


def test_isolated_molecules_fp64(isolated, isolated_ref):
    sv = solve(isolated, "fp64")
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    worst = max(rel(dc[J], isolated_ref.Dcols[J]) for J in range(isolated.nmol))
    say(f"isolated fp64: worst Dcols rel-F {worst:.3e}")
    assert worst <= 1e-10
    assert np.allclose(st["energy_KD"], isolated_ref.E, rtol=0, atol=1e-10)
    assert np.allclose(st["trace_SD"], isolated_ref.N, rtol=0, atol=1e-10)


@pytest.mark.parametrize("prec,sym,apply32", [("fp16", 1, 0), ("fp16", 0, 0), ("bf16", 1, 0), ("fp16", 1, 1),
                                              ("bf16", 1, 1)])
def test_isolated_molecules_mixed(isolated, isolated_ref, prec, sym, apply32):
    # one 64-row tile per submatrix; apply32: the FP64 factor applied in FP32
    # (on the symmetric route as split FP16 products)
    from paper_2104_08245_amd import _lib as L
    kw = {"inverse": L.INV_CHOLESKY_APPLY_FP32} if apply32 else {}
    sv = solve(isolated, prec, sym_sign=sym, **kw)
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], isolated_ref.Dcols[J]) for J in range(isolated.nmol)])
    de = np.abs(st["energy_KD"] - isolated_ref.E)
    say(f"isolated {prec} sym={sym} apply32={apply32}: Dcols max {errs.max():.3e}; |dE| max {de.max():.3e}")
    assert errs.max() <= MIXED[prec]["dcols"] and de.max() <= MIXED[prec]["energy"]


@pytest.fixture(scope="module")
def largest():
    from paper_2104_08245_amd import _lib as L
    s = synth.water_cube(501, 2.2, config_id=111)
    assert s.K.nnzb == s.nmol * s.nmol and 6 * s.nmol <= L.MAX_ROWS
    return s


@pytest.fixture(scope="module")
def exact(largest):
    Kd, Sd = o.dense(largest.K), o.dense(largest.S)
    w, C = sla.eigh(Kd, Sd)
    Co = C[:, w < 0.0]
    D = Co @ Co.T
    bs = largest.K.bs
    E = np.array([np.trace(Kd[bs * J:bs * J + bs, :] @ D[:, bs * J:bs * J + bs]) for J in range(largest.nmol)])
    say(f"exact full cell: n {Kd.shape[0]}, occupied {Co.shape[1]}")
    return D, E


def check_largest(sv, largest, exact, tol_d, tol_e, tag):
    D, E = exact
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    bs = largest.K.bs
    errs = np.array([rel(dc[J], D[:, bs * J:bs * J + bs]) for J in range(largest.nmol)])
    de = np.abs(st["energy_KD"] - E)
    say(f"largest {tag}: Dcols rel-F max {errs.max():.3e} mean {errs.mean():.3e}; |dE| max {de.max():.3e} "
        f"mean {de.mean():.3e}; iterations {st['iters'].min()}..{st['iters'].max()}")
    assert errs.max() <= tol_d and de.max() <= tol_e


def test_largest_submatrix_fp64(largest, exact):
    sv = solve(largest, "fp64", ws_budget=48 << 30)
    assert sv.plan.info()["nchunks"] >= 2
    check_largest(sv, largest, exact, 1e-10, 1e-9, "fp64")


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_largest_submatrix_mixed(largest, exact, prec):
    from paper_2104_08245_amd import _lib as L
    sv = solve(largest, prec, sym_sign=1, inverse=L.INV_CHOLESKY_APPLY_FP32, ws_budget=48 << 30)
    check_largest(sv, largest, exact, MIXED[prec]["dcols"], MIXED[prec]["energy"], prec)
