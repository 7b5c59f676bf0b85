"""Global checks of an assembled D (paper_2104_08245_amd.diagnostics), pinned
on the CPU by the oracle's D:

- full cell (every submatrix is the whole matrix): NOLSM gives the exact
  density matrix, so D S D = D, D = D^T and Tr(D S) = 4 per molecule up to
  rounding;
- the 64-molecule box (truncated submatrices): the idempotency floor of the
  FP64 method is well above rounding, D is not symmetric, the trace stays 4
  per molecule (the generator's gap), and the probe estimate of
  ||D S D - D||_F agrees with the exact value within its statistical error.
"""
import numpy as np

import synth
from oracle import nolsm as o
from paper_2104_08245_amd import diagnostics as dg


def assembled(system):
    r = o.nolsm(system)
    p = r.plan
    nb, bs = system.K.nb, system.K.bs
    D = dg.block_csr(nb, bs, p["D_row_ptr"], p["D_col_idx"], r.D_val)
    S = dg.block_csr(nb, bs, system.S.row_ptr, system.S.col_idx, system.S.val)
    return D, S


def test_full_cell_density_is_an_exact_projector():
    s = synth.water_cube(16, 0.7, config_id=102)
    D, S = assembled(s)
    c = dg.density_checks(D, S, s.nmol)
    assert c["idempotency"] < 1e-11
    assert c["asymmetry"] < 1e-11
    assert abs(c["trace_DS_per_molecule"] - 4.0) < 1e-10


def test_truncated_box_floor_and_probe_estimate(box64):
    D, S = assembled(box64)
    exact = dg.density_checks(D, S, box64.nmol)
    assert 1e-6 < exact["idempotency"] < 0.1
    assert exact["asymmetry"] > 1e-6
    assert abs(exact["trace_DS_per_molecule"] - 4.0) < 1e-5
    est = dg.density_checks(D, S, box64.nmol, probes=64, seed=3)
    # relative standard error of the estimate ~ 1/sqrt(2 * 64) = 0.09
    assert abs(est["idempotency"] / exact["idempotency"] - 1.0) < 0.3
    assert est["asymmetry"] == exact["asymmetry"]
