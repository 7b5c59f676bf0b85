"""The symmetric sign iteration (option sym_sign) vs the CPU oracle, through
the C ABI.

With S_J = L L^T, A_J - mu I = L^-T (L^-1 K_J L^-T - mu I) L^T, so
sign(A_J) = L^-T sign(A~) L^T with A~ = L^-1 K_J L^-T - mu I symmetric, and
the owned columns of D are L^-T (y - sign(A~) y) / 2 with y = L^-1 E_cJ: the
same D as the oracle's definition (Eq. purification_submatrix). The 16-bit
iteration on A~ has the same spectrum and the same FP16/BF16 floor as the one
on A_J, so the mixed bounds of the per-molecule path apply unchanged. Outside
the spectrum the sign is -I or +I after a few steps and the result is exact to
the factor's precision, which pins the setup (A~, y) and the final L^-T solve
tightly.
"""
import sys

import numpy as np
import pytest

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
def ref1(box64):
    return o.nolsm(box64)


def solve(system, prec, mu=None, **kw):
    from paper_2104_08245_amd import Solver
    import torch
    say(f"[gpu] symmetric solve prec={prec} nmol={system.nmol} mu={mu} {kw}")
    sv = Solver(system, prec=prec, device="cuda:0", sym_sign=1, **kw)
    sv.run(mu=mu)
    torch.cuda.synchronize()
    return sv


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def check_mixed(sv, ref, nmol, prec, tag):
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref.Dcols[J]) for J in range(nmol)])
    de = np.abs(st["energy_KD"] - ref.E)
    say(f"{tag}: Dcols rel-F max {errs.max():.3e} mean {errs.mean():.3e}; |dE_J| max {de.max():.3e}; "
        f"iters {st['iters'].min()}..{st['iters'].max()}")
    assert errs.max() <= MIXED[prec]["dcols"]
    assert de.max() <= MIXED[prec]["energy"]
    return st


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_symmetric_within_stated_error(torch, box64, ref1, prec):
    from paper_2104_08245_amd import Solver
    st = check_mixed(solve(box64, prec), ref1, box64.nmol, prec, f"{prec} symmetric")
    # same spectrum, same scale rule, same stopping rule: the iteration
    # counts stay those of the iteration on A_J, up to where each run's
    # 16-bit rounding lets the residual cross the switch point (BF16: within 2)
    on_a = Solver(box64, prec=prec, device="cuda:0")
    on_a.run()
    torch.cuda.synchronize()
    assert np.all(np.abs(st["iters"] - on_a.host_stats()["iters"]) <= 2)


@pytest.mark.parametrize("subst_fp32", [0, 1])
def test_symmetric_on_fp32_factor(torch, box64, ref1, subst_fp32):
    from paper_2104_08245_amd import _lib as L
    check_mixed(solve(box64, "fp16", inverse=L.INV_CHOLESKY_FP32, subst_fp32=subst_fp32), ref1, box64.nmol,
                "fp16", f"fp16 symmetric, FP32 factor, subst_fp32={subst_fp32}")


@pytest.mark.parametrize("prec,subst_fp32", [("fp16", 0), ("bf16", 0), ("fp16", 1), ("bf16", 1)])
def test_symmetric_on_fp64_factor_applied_in_fp32(torch, box64, ref1, prec, subst_fp32):
    # the FP32 substitutions as split FP16 products (default) or on the FP32
    # matrix cores (subst_fp32)
    from paper_2104_08245_amd import _lib as L
    check_mixed(solve(box64, prec, inverse=L.INV_CHOLESKY_APPLY_FP32, subst_fp32=subst_fp32), ref1, box64.nmol,
                prec, f"{prec} symmetric, FP64 factor applied in FP32, subst_fp32={subst_fp32}")


def test_fp64_factor_applied_in_fp32_outside_spectrum(torch, box64):
    # sign = -I above the spectrum: Dcols = S_J^-1 E_cJ, formed through the
    # FP32 copy of the factor (y = L^-1 E) and the FP64 factor (L^-T); the
    # FP32 application costs about kappa(L) 2^-24 relative (split FP16
    # products, the symmetric route's default: about kappa(L) 2^-22)
    from paper_2104_08245_amd import _lib as L
    from paper_2104_08245_amd import Solver
    Js = list(range(0, box64.nmol, 7))
    hi = o.nolsm(box64, mu=50.0, molecules=Js)
    for sym, subst_fp32 in ((1, 0), (1, 1), (0, 0)):
        sv = Solver(box64, prec="fp16", device="cuda:0", sym_sign=sym, inverse=L.INV_CHOLESKY_APPLY_FP32,
                    subst_fp32=subst_fp32)
        sv.run(mu=50.0)
        torch.cuda.synchronize()
        dc = sv.host_dcols()
        worst = max(rel(dc[J], hi.Dcols[J]) for J in Js)
        say(f"FP64 factor applied in FP32, sym={sym}, subst_fp32={subst_fp32}, mu=50: worst rel-F {worst:.3e}")
        assert worst <= 1e-5


def test_symmetric_nonzero_mu(torch, box64):
    ref = o.nolsm(box64, mu=0.25)
    check_mixed(solve(box64, "fp16", mu=0.25), ref, box64.nmol, "fp16", "fp16 symmetric mu=0.25")


def test_symmetric_outside_spectrum_is_exact(torch, box64):
    # mu above the spectrum: sign = -I and Dcols = S_J^-1 E_cJ; the FP32
    # finishing leaves ~1e-7, so the setup and the L^-T solve are held to 1e-5
    Js = list(range(0, box64.nmol, 7))
    hi = o.nolsm(box64, mu=50.0, molecules=Js)
    sv = solve(box64, "fp16", mu=50.0)
    dc = sv.host_dcols()
    worst = max(rel(dc[J], hi.Dcols[J]) for J in Js)
    say("symmetric mu=50 worst rel-F", worst)
    assert worst <= 1e-5
    sv.run(mu=-50.0)
    torch.cuda.synchronize()
    assert np.abs(sv.Dcols.cpu().numpy()).max() <= 1e-5 * max(np.abs(d).max() for d in dc)


@pytest.mark.parametrize("route", ["cholesky", "apply_fp32"])
def test_symmetric_combined(torch, box64, route):
    # combined submatrices (several owned molecules, larger n), with the FP64
    # application and with the FP32 one as split FP16 products
    from paper_2104_08245_amd import _lib as L
    inv = {"cholesky": L.INV_CHOLESKY, "apply_fp32": L.INV_CHOLESKY_APPLY_FP32}[route]
    sv = solve(box64, "fp16", combine=True, inverse=inv)
    ref = o.nolsm_groups(box64, sv.plan.groups())
    check_mixed(sv, ref, box64.nmol, "fp16", f"fp16 symmetric combined, {route}")


@pytest.mark.parametrize("prec", ["fp16"])
def test_symmetric_schedules_chunks_and_replays_bit_identical(torch, box64, prec):
    from paper_2104_08245_amd import Solver, _lib as L
    base = solve(box64, prec, sched=L.SCHED_STREAM)
    ref = base.Dcols.cpu().numpy()
    for kw in (dict(sched=L.SCHED_PERSISTENT), dict(sched=L.SCHED_PER_BUCKET),
               dict(ws_bytes=base.plan.info()["ws_full_bytes"] // 3 + 4096)):
        other = solve(box64, prec, **kw)
        assert np.array_equal(other.Dcols.cpu().numpy(), ref), kw
    sv = Solver(box64, prec=prec, device="cuda:0", sym_sign=1, sched=L.SCHED_GRAPH)
    s = torch.cuda.Stream()
    for rep in range(3):
        say(f"[gpu] symmetric graph replay {rep}")
        sv.Dcols.zero_()
        torch.cuda.synchronize()
        sv.run(stream=s)
        s.synchronize()
        assert np.array_equal(sv.Dcols.cpu().numpy(), ref), rep


def test_symmetric_not_spd_flagged(torch, box64, ref1):
    sv = solve(box64, "fp16", debug_poison_mol=5)
    st = sv.host_stats()
    assert st["status"][5] != 0
    assert np.all(np.delete(st["status"], 5) == 0)


def test_symmetric_rejects_outputs_defined_on_a(torch, box64):
    from paper_2104_08245_amd import Solver, NolsmError, _lib as L
    sv = Solver(box64, prec="fp16", device="cuda:0", sym_sign=1)
    sv.want_w()
    with pytest.raises(NolsmError) as e:
        sv.run()
    assert e.value.code == L.E_ARG


@pytest.mark.parametrize("sym", [1, 0])
def test_fused_finishing_matches_row_kernel(torch, box64, ref1, sym):
    # the FP16 finishing products on the matrix cores (P [h | l], the input
    # split into FP16 high and low parts) against the row-streaming FP32
    # vector kernel on the same iterate: both FP32-accurate, so they agree far
    # below the 16-bit floor; both stay within the stated bounds of the oracle
    from paper_2104_08245_amd import Solver
    out = {}
    for rows in (0, 1):
        sv = Solver(box64, prec="fp16", device="cuda:0", sym_sign=sym, finish_rows=rows)
        sv.run()
        torch.cuda.synchronize()
        st = sv.host_stats()
        assert np.all(st["status"] == 0) and np.all(st["iters_fp32"] == 2)
        out[rows] = (sv.host_dcols(), st)
    (d0, s0), (d1, s1) = out[0], out[1]
    assert np.array_equal(s0["iters"], s1["iters"])
    diff = max(rel(d0[J], d1[J]) for J in range(box64.nmol))
    dE = np.abs(s0["energy_KD"] - s1["energy_KD"]).max()
    say(f"fused vs row finishing (sym={sym}): worst Dcols rel-F {diff:.3e}, max |dE| {dE:.3e}")
    assert diff <= 2e-5 and dE <= 1e-5
    errs = np.array([rel(d0[J], ref1.Dcols[J]) for J in range(box64.nmol)])
    assert errs.max() <= MIXED["fp16"]["dcols"]
    assert np.abs(s0["energy_KD"] - ref1.E).max() <= MIXED["fp16"]["energy"]
