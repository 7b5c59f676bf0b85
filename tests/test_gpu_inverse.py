"""The coupled Newton-Schulz route to T_J(S)^-1 (Eq. inv1-inv3, FP16 / BF16 on
the matrix cores) vs the CPU oracle, through the C ABI.

In exact arithmetic both routes give the same D (pinned on the CPU by
test_i4_density_matrix_equals_cholesky_route), so the GPU result is held to
the FP64 oracle with bounds for 16-bit operands. The inverse stops at the
16-bit floor of ||I - Z Y||_F, which leaves S^-1, Y_J and A_J with a relative
error of a few 1e-3 in FP16 (unit roundoff 2^-11 times the growth of the
iteration); the sign of A_J amplifies the error of A_J by about 1 / gap
(gap ~ 0.23 for this generator, a factor ~4), so Dcols is held to 3e-2
relative in FP16 and 8x that in BF16 (3 fewer mantissa bits): 2.5e-1. The
energies follow from Dcols: |dE_J| = |tr(K_J[cJ, :] dDcols_J)| <=
||K_J[cJ, :]||_F ||dDcols_J||_F, checked with the same relative bound, and
held besides to an absolute per-molecule bound: measured on the 64-molecule
box, max |dE_J| is 0.168 (mean 0.037) in FP16 and 0.951 (mean 0.308) in
BF16, about a hundred times the Cholesky route's; the bounds are twice the
measured maxima and means.
"""
import sys

import numpy as np
import pytest

from oracle import nolsm as o

pytestmark = pytest.mark.gpu

BOUNDS = {"fp16": 3e-2, "bf16": 2.5e-1}
ENERGY_ABS = {"fp16": dict(max=0.34, mean=0.074), "bf16": dict(max=1.9, mean=0.62)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def ref1(box64):
    return o.nolsm(box64)


def solve(system, prec, **kw):
    from paper_2104_08245_amd import Solver, _lib as L
    import torch
    say(f"[gpu] coupled-NS inverse prec={prec} nmol={system.nmol} {kw}")
    sv = Solver(system, prec=prec, device="cuda:0", inverse=L.INV_COUPLED_NS, **kw)
    sv.run()
    torch.cuda.synchronize()
    return sv


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_coupled_inverse_route_matches_oracle(torch, box64, ref1, prec):
    sv = solve(box64, prec)
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    assert np.all((st["iters_inv"] >= 5) & (st["iters_inv"] <= 30))
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref1.Dcols[J]) for J in range(box64.nmol)])
    dE = np.abs(st["energy_KD"] - ref1.E)
    say(f"{prec} coupled-NS route: Dcols rel-F max {errs.max():.3e} mean {errs.mean():.3e}; "
        f"|dE| max {dE.max():.3e} mean {dE.mean():.3e}; inverse iterations "
        f"{st['iters_inv'].min()}..{st['iters_inv'].max()}")
    assert errs.max() <= BOUNDS[prec]
    assert dE.max() <= ENERGY_ABS[prec]["max"] and dE.mean() <= ENERGY_ABS[prec]["mean"]
    for J in range(box64.nmol):
        KJ, _, _, p = o.submatrix(box64, J)
        krows = KJ[6 * p:6 * p + 6, :]
        assert dE[J] <= BOUNDS[prec] * np.linalg.norm(krows) * np.linalg.norm(ref1.Dcols[J])


def test_cholesky_route_reports_no_inverse_iterations(torch, box64):
    from paper_2104_08245_amd import Solver
    import torch as T
    sv = Solver(box64, prec="fp16", device="cuda:0")
    sv.run()
    T.cuda.synchronize()
    assert np.all(sv.host_stats()["iters_inv"] == 0)


def test_coupled_inverse_flags_indefinite_overlap(torch, box64, ref1):
    # S_J with a negative pivot: the scaled iteration has an eigenvalue of
    # c S_J below 0 and diverges, which marks the molecule NOT_SPD: its sign
    # iteration is skipped, its columns stay zero, its traces are zero, and
    # the synchronous mode reports E_NOT_SPD (as on the Cholesky route)
    from paper_2104_08245_amd import NolsmError, _lib as L
    sv = solve(box64, "fp16", debug_poison_mol=3)
    st = sv.host_stats()
    assert st["status"][3] == L.MOL_NOT_SPD
    ok = np.arange(box64.nmol) != 3
    assert np.all(st["status"][ok] == 0)
    dc = sv.host_dcols()
    assert np.all(dc[3] == 0)
    assert st["trace_SD"][3] == 0 and st["energy_KD"][3] == 0
    assert rel(dc[4], ref1.Dcols[4]) <= BOUNDS["fp16"]
    sv.set_opts(sync_errors=1)
    with pytest.raises(NolsmError) as e:
        sv.run()
    assert e.value.code == L.E_NOT_SPD


def test_coupled_inverse_route_nonzero_mu(torch, box64):
    from paper_2104_08245_amd import Solver, _lib as L
    ref = o.nolsm(box64, mu=0.25)
    sv = Solver(box64, prec="fp16", device="cuda:0", inverse=L.INV_COUPLED_NS)
    sv.run(mu=0.25)
    torch.cuda.synchronize()
    assert np.all(sv.host_stats()["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref.Dcols[J]) for J in range(box64.nmol)])
    say(f"fp16 coupled-NS mu=0.25: Dcols rel-F max {errs.max():.3e}")
    assert errs.max() <= BOUNDS["fp16"]
