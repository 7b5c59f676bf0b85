"""NOLSM on combined submatrices (Sec. III-B, submatrix combination) on the
GPU vs the CPU oracle on the same groups, through the C ABI.

The groups come from the library's plan (their equality with the oracle's
heuristic is a CPU test); the oracle then builds each group's submatrix on the
union of its molecules' row blocks and cuts every owned molecule's columns
back to N(J). FP64 is held to 1e-10 relative like the per-molecule path. The
16-bit paths run the sign iteration on larger submatrices (up to 2-3x the rows
of one molecule) whose spectra stay in the same interval, so the per-molecule
bounds of the mixed path apply unchanged. In a full cell every submatrix is
the whole matrix, so combined and uncombined runs must agree to rounding.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import nolsm as o

pytestmark = pytest.mark.gpu

MIXED = {"fp16": dict(dcols=5e-3, energy=1e-3), "bf16": dict(dcols=4e-2, energy=1e-2)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def full_cell():
    return synth.water_cube(16, 0.7, config_id=102)


def solve(system, prec, **kw):
    from paper_2104_08245_amd import Solver
    import torch
    say(f"[gpu] combined solve prec={prec} nmol={system.nmol} opts={kw}")
    sv = Solver(system, prec=prec, device="cuda:0", combine=True, **kw)
    sv.run()
    torch.cuda.synchronize()
    return sv


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def oracle_on(system, sv):
    g = sv.plan.groups()
    return o.nolsm_groups(system, g), g


def test_fp64_combined_matches_oracle_box64(torch, box64):
    sv = solve(box64, "fp64")
    ref, g = oracle_on(box64, sv)
    say(f"box64: {len(g[0]) - 1} groups for {box64.nmol} molecules, "
        f"largest owns {np.diff(g[2]).max()}")
    assert len(g[0]) - 1 < box64.nmol
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    worst = max(rel(dc[J], ref.Dcols[J]) for J in range(box64.nmol))
    say("fp64 combined worst per-molecule rel-F", worst)
    assert worst <= 1e-10
    assert rel(sv.host_D(), ref.D_val) <= 1e-10
    assert np.allclose(st["trace_SD"], ref.N, rtol=0, atol=1e-10)
    assert np.allclose(st["energy_KD"], ref.E, rtol=0, atol=1e-10)
    assert np.all(np.abs(st["iters"] - ref.iters) <= 1)


def test_fp64_full_cell_groups_fill_the_tile(torch, full_cell):
    sv = solve(full_cell, "fp64")
    ref, g = oracle_on(full_cell, sv)
    assert sorted(np.diff(g[2]).tolist()) == [6, 10]
    dc = sv.host_dcols()
    worst = max(rel(dc[J], ref.Dcols[J]) for J in range(full_cell.nmol))
    say("full cell fp64 combined worst rel-F", worst)
    assert worst <= 1e-10
    assert rel(sv.host_D(), ref.D_val) <= 1e-10


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_combined_within_stated_error(torch, box64, prec):
    sv = solve(box64, prec)
    ref, _ = oracle_on(box64, sv)
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref.Dcols[J]) for J in range(box64.nmol)])
    de = np.abs(st["energy_KD"] - ref.E)
    say(f"{prec} combined: Dcols rel-F max {errs.max():.3e} mean {errs.mean():.3e}; "
        f"|dE_J| max {de.max():.3e}")
    assert errs.max() <= MIXED[prec]["dcols"]
    assert de.max() <= MIXED[prec]["energy"]


def test_full_cell_combined_equals_uncombined_with_w(torch, full_cell):
    from paper_2104_08245_amd import Solver
    runs = []
    for comb in (False, True):
        sv = Solver(full_cell, prec="fp64", device="cuda:0", combine=comb)
        sv.want_w()
        sv.run()
        torch.cuda.synchronize()
        runs.append((sv.host_dcols(), sv.host_dcols("W")))
    for J in range(full_cell.nmol):
        assert rel(runs[1][0][J], runs[0][0][J]) <= 1e-10
        assert rel(runs[1][1][J], runs[0][1][J]) <= 1e-9


def test_combined_coupled_inverse_route(torch, box64):
    # bounds of the 16-bit inverse route (derived with the per-molecule test)
    from paper_2104_08245_amd import _lib as L
    sv = solve(box64, "fp16", inverse=L.INV_COUPLED_NS)
    ref, _ = oracle_on(box64, sv)
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref.Dcols[J]) for J in range(box64.nmol)])
    say(f"fp16 combined coupled-NS: Dcols rel-F max {errs.max():.3e}")
    assert errs.max() <= 3e-2


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_combined_chunked_and_replayed_bit_identical(torch, box64, prec):
    from paper_2104_08245_amd import Solver, _lib as L
    one = solve(box64, prec)
    ref = one.Dcols.cpu().numpy()
    full = one.plan.info()["ws_full_bytes"]
    many = solve(box64, prec, ws_bytes=full // 3 + 4096)
    assert many.plan.info()["nchunks"] >= 3
    assert np.array_equal(many.Dcols.cpu().numpy(), ref)
    assert np.array_equal(many.D.cpu().numpy(), one.D.cpu().numpy())
    sv = Solver(box64, prec=prec, device="cuda:0", combine=True, sched=L.SCHED_GRAPH)
    s = torch.cuda.Stream()
    for rep in range(3):
        say(f"[gpu] combined graph replay {rep} prec={prec}")
        sv.Dcols.zero_()
        torch.cuda.synchronize()
        sv.run(stream=s)
        s.synchronize()
        assert np.array_equal(sv.Dcols.cpu().numpy(), ref), rep


def test_not_spd_marks_every_owned_molecule(torch, box64):
    sv = solve(box64, "fp64", debug_poison_mol=5)
    g = sv.plan.groups()
    grp = int(np.searchsorted(g[2], np.flatnonzero(g[3] == 5)[0], side="right") - 1)
    owned = set(g[3][g[2][grp]:g[2][grp + 1]].tolist())
    st = sv.host_stats()
    say(f"poisoned molecule 5 sits in a group owning {sorted(owned)}")
    for J in range(box64.nmol):
        assert (st["status"][J] != 0) == (J in owned)


def test_fp64_combined_nonzero_mu(torch, box64):
    sv = solve(box64, "fp64")
    g = sv.plan.groups()
    ref = o.nolsm_groups(box64, g, mu=0.25)
    sv.run(mu=0.25)
    torch.cuda.synchronize()
    dc = sv.host_dcols()
    worst = max(rel(dc[J], ref.Dcols[J]) for J in range(box64.nmol))
    say("fp64 combined mu=0.25 worst rel-F", worst)
    assert worst <= 1e-10
