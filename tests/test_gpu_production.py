"""The benchmarked path at production size, and inputs whose K and S patterns
differ, against the CPU oracle through the C ABI.

The bench runs the 16-bit sign iteration on the symmetric similar matrix
(sym_sign), the FP64 Cholesky factor applied through its FP32 copy, the
graph schedule on a side stream and several chunks of submatrices with n_J
516-708. The 4,096-molecule cube at r_c 0.9 nm
has the same submatrix sizes (n_J 534-696: 5-6 NS tile rows of 128 with the
mirrored off-diagonal tiles, 9-11 row blocks of the right solve), so it is
solved here exactly as the bench solves its batch, and a seeded sample of
molecules (with the smallest and the largest submatrix) is compared element
by element with the FP64 oracle at the stated mixed-precision bounds.

Unequal patterns (Sec. III-B.2: the submatrix rows are the union of the rows
where H_0 or S is stored): K truncated at a smaller cutoff than S, and the
reverse, so that the gather meets blocks present in one matrix and absent in
the other; FP64 is held to 1e-10, the mixed path to its stated bounds.
"""
import hashlib
import os
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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def cube():
    return synth.make_config(2)


@pytest.fixture(scope="module")
def sample(cube):
    m = np.diff(cube.K.row_ptr)
    rng = np.random.default_rng(2104)
    mols = set(rng.choice(cube.nmol, 30, replace=False).tolist())
    mols |= {int(np.argmin(m)), int(np.argmax(m))}
    return sorted(mols)


@pytest.fixture(scope="module")
def ref(cube, sample):
    say(f"[cpu] oracle on {len(sample)} molecules of the 4096-molecule cube")
    return {J: o.solve_molecule(cube, J) for J in sample}


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube4096_traces.npz")


def golden_traces(system):
    """The oracle's N_J and E_J of every molecule of the 4,096-molecule cube
    (tests/golden/make_cube4096_traces.py), checked to belong to `system`."""
    g = np.load(GOLDEN)
    h = hashlib.sha256()
    for a in (system.K.row_ptr, system.K.col_idx, system.K.val, system.S.row_ptr, system.S.col_idx,
              system.S.val):
        h.update(np.ascontiguousarray(a).tobytes())
    assert str(g["digest"]) == h.hexdigest(), "golden traces were written for another system"
    assert np.all(g["status"] == 0)
    return {"N": g["N"], "E": g["E"]}


def full_workspace(system, **kw):
    """Workspace bytes of the whole batch in one chunk (host-side plan only)."""
    from paper_2104_08245_amd import Plan, _lib as L
    K, S = system.K, system.S
    p = Plan(K.nb, K.bs, K.row_ptr, K.col_idx, S.row_ptr, S.col_idx)
    p.configure(L.default_opts(**kw), 1 << 44)
    return p.info()["ws_full_bytes"]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_bench_path_at_production_size(torch, cube, sample, ref, prec):
    from paper_2104_08245_amd import Solver, _lib as L
    kw = dict(prec=prec, sym_sign=1, inverse=L.INV_CHOLESKY_APPLY_FP32, sched=L.SCHED_GRAPH)
    ws = full_workspace(cube, **kw) // 3 + (1 << 20)
    sv = Solver(cube, device="cuda:0", ws_bytes=ws, **kw)
    inf = sv.plan.info()
    n = 6 * np.diff(cube.K.row_ptr)
    say(f"[gpu] {prec} symmetric, graph on a side stream, {inf['nchunks']} chunks, n {n.min()}..{n.max()}")
    assert inf["nchunks"] >= 2
    assert n.min() >= 516 and n.max() <= 708
    s = torch.cuda.Stream()
    runs = []
    for rep in range(2):
        sv.Dcols.zero_()
        torch.cuda.synchronize()
        sv.run(stream=s)
        s.synchronize()
        runs.append(sv.Dcols.cpu().numpy())
    # the captured graph replays bit-identically
    assert np.array_equal(runs[0], runs[1])
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    assert np.all(st["iters_fp32"] == 2)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref[J].Dcols) for J in sample])
    de = np.array([abs(st["energy_KD"][J] - ref[J].E_J) for J in sample])
    dn = np.array([abs(st["trace_SD"][J] - ref[J].N_J) for J in sample])
    say(f"{prec} production size, {len(sample)} molecules: Dcols rel-F max {errs.max():.3e} mean "
        f"{errs.mean():.3e}; |dE_J| max {de.max():.3e} mean {de.mean():.3e}; |dN_J| max {dn.max():.3e}; "
        f"iters {st['iters'].min()}..{st['iters'].max()}")
    assert errs.max() <= MIXED[prec]["dcols"]
    assert de.max() <= MIXED[prec]["energy"]
    # every molecule at full size: N_J and E_J against the oracle's values
    # for all 4,096 molecules (tests/golden, written by its script from the
    # oracle alone); the truncation makes N_J differ from 4 per molecule,
    # the oracle's sum over molecules stays at 4 per molecule
    gold = golden_traces(cube)
    dE = np.abs(st["energy_KD"] - gold["E"])
    dN = np.abs(st["trace_SD"] - gold["N"])
    say(f"{prec} all {cube.nmol} molecules vs oracle: |dE_J| max {dE.max():.3e} mean {dE.mean():.3e}; "
        f"|dN_J| max {dN.max():.3e}; oracle N_J {gold['N'].min():.4f}..{gold['N'].max():.4f}")
    assert dE.max() <= MIXED[prec]["energy"]
    assert dN.max() <= MIXED[prec]["energy"]
    assert abs(st["trace_SD"].sum() - gold["N"].sum()) / cube.nmol <= MIXED[prec]["energy"]


@pytest.fixture(scope="module", params=["k_smaller", "s_smaller"])
def unequal(request, box64):
    if request.param == "k_smaller":
        s = synth.two_cutoffs(box64, r_k=0.45)   # pat(S) strictly contains pat(K)
    else:
        s = synth.two_cutoffs(box64, r_s=0.45)   # pat(K) strictly contains pat(S)
    assert s.K.nnzb != s.S.nnzb
    return request.param, s


def test_unequal_patterns_fp64(torch, unequal):
    from paper_2104_08245_amd import Solver
    name, s = unequal
    ref = o.nolsm(s)
    sv = Solver(s, prec="fp64", device="cuda:0")
    sv.run()
    torch.cuda.synchronize()
    st = sv.host_stats()
    assert np.all(st["status"] == 0) and np.all(ref.status == 0)
    dc = sv.host_dcols()
    worst = max(rel(dc[J], ref.Dcols[J]) for J in range(s.nmol))
    say(f"unequal patterns ({name}, K {s.K.nnzb} / S {s.S.nnzb} blocks): FP64 worst rel-F {worst:.3e}")
    assert worst <= 1e-10
    assert rel(sv.host_D(), ref.D_val) <= 1e-10
    assert np.allclose(st["trace_SD"], ref.N, rtol=0, atol=1e-10)
    assert np.allclose(st["energy_KD"], ref.E, rtol=0, atol=1e-10)


@pytest.mark.parametrize("sym", [0, 1])
def test_unequal_patterns_fp16(torch, unequal, sym):
    from paper_2104_08245_amd import Solver
    name, s = unequal
    ref = o.nolsm(s)
    sv = Solver(s, prec="fp16", device="cuda:0", sym_sign=sym)
    sv.run()
    torch.cuda.synchronize()
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([rel(dc[J], ref.Dcols[J]) for J in range(s.nmol)])
    de = np.abs(st["energy_KD"] - ref.E)
    say(f"unequal patterns ({name}) fp16 sym={sym}: Dcols rel-F max {errs.max():.3e}; |dE_J| max {de.max():.3e}")
    assert errs.max() <= MIXED["fp16"]["dcols"]
    assert de.max() <= MIXED["fp16"]["energy"]
