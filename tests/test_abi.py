"""The C ABI on the CPU: the library loads, exports every declared symbol, its
struct layouts match the binding, and the plan (pure host work) equals the
oracle's merge exactly. No kernel is launched here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from oracle import nolsm as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nolsm.h")


@pytest.fixture(scope="module")
def L():
    from paper_2104_08245_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libnolsm.so not built (run __graft_entry__.build())")
    return _lib


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nolsm_[A-Za-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_struct_layouts_match_header(L, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "nolsm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(nolsm_pattern), sizeof(nolsm_solve_opts), sizeof(nolsm_mol_stats), sizeof(nolsm_plan_sizes), sizeof(nolsm_profile));
  printf("%zu %zu %zu %zu %zu\n", offsetof(nolsm_solve_opts, d_mlp), offsetof(nolsm_solve_opts, sched),
         offsetof(nolsm_solve_opts, d_features), offsetof(nolsm_solve_opts, debug_poison_mol),
         offsetof(nolsm_plan_sizes, ws_full_bytes));
  return 0; }
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    want = [C.sizeof(L.Pattern), C.sizeof(L.SolveOpts), C.sizeof(L.MolStats), C.sizeof(L.PlanSizes),
            C.sizeof(L.Profile),
            L.SolveOpts.d_mlp.offset, L.SolveOpts.sched.offset, L.SolveOpts.d_features.offset,
            L.SolveOpts.debug_poison_mol.offset, L.PlanSizes.ws_full_bytes.offset]
    assert got == want
    assert np.dtype(L.MOLSTATS_DTYPE).itemsize == C.sizeof(L.MolStats)


def test_plan_equals_oracle_merge(L, box64):
    from paper_2104_08245_amd import Plan
    s = box64
    p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    ex = p.export()
    ref = o.plan_arrays(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    for k in ("sub_ptr", "sub_blk", "self_pos", "D_row_ptr", "D_col_idx", "scatter_pos"):
        assert np.array_equal(ex[k], ref[k]), k
    inf = p.info()
    m = np.diff(ref["sub_ptr"])
    assert inf["sum_m"] == m.sum() and inf["m_min"] == m.min() and inf["m_max"] == m.max()
    assert inf["sum_n3"] == pytest.approx(((6 * m) ** 3).sum())


@pytest.mark.parametrize("kw", [dict(r_k=0.45), dict(r_s=0.45)])
def test_plan_equals_oracle_merge_two_cutoffs(L, box64, kw):
    # K and S truncated at different cutoffs: the plan's merge of the two
    # generated patterns equals the oracle's, and N(J) is the larger pattern
    import synth
    from paper_2104_08245_amd import Plan
    s = synth.two_cutoffs(box64, **kw)
    p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    ex = p.export()
    ref = o.plan_arrays(s.K.nb, s.K.row_ptr, s.K.col_idx, s.S.row_ptr, s.S.col_idx)
    for k in ("sub_ptr", "sub_blk", "self_pos", "D_row_ptr", "D_col_idx", "scatter_pos"):
        assert np.array_equal(ex[k], ref[k]), k
    big = s.S if "r_k" in kw else s.K
    assert np.array_equal(ex["sub_ptr"], big.row_ptr) and np.array_equal(ex["sub_blk"], big.col_idx)


def _random_pair_patterns(rng, nb, pk, ps):
    def sym(p):
        A = rng.random((nb, nb)) < p
        A = A | A.T | np.eye(nb, dtype=bool)
        rp = np.concatenate([[0], np.cumsum(A.sum(1))]).astype(np.int32)
        ci = np.concatenate([np.nonzero(A[i])[0] for i in range(nb)]).astype(np.int32)
        return rp, ci
    return sym(pk), sym(ps)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_merges_different_patterns(L, seed):
    from paper_2104_08245_amd import Plan
    rng = np.random.default_rng(seed)
    nb = 37
    (krp, kci), (srp, sci) = _random_pair_patterns(rng, nb, 0.08, 0.12)
    p = Plan(nb, 6, krp, kci, srp, sci)
    ex = p.export()
    ref = o.plan_arrays(nb, krp, kci, srp, sci)
    for k in ("sub_ptr", "sub_blk", "self_pos", "D_row_ptr", "D_col_idx", "scatter_pos"):
        assert np.array_equal(ex[k], ref[k]), k


@pytest.mark.parametrize("case", ["unsorted", "no_diag", "asym", "range", "rowptr"])
def test_malformed_patterns_rejected(L, case):
    from paper_2104_08245_amd import Plan, NolsmError
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    if case == "unsorted":
        ci = np.array([1, 0, 0, 1], np.int32)
    elif case == "no_diag":
        rp, ci = np.array([0, 1, 3], np.int32), np.array([1, 0, 1], np.int32)
    elif case == "asym":
        rp, ci = np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32)
    elif case == "range":
        ci = np.array([0, 2, 0, 1], np.int32)
    elif case == "rowptr":
        rp = np.array([0, 3, 4], np.int32)
    with pytest.raises(NolsmError) as e:
        Plan(2, 6, rp, ci)
    assert e.value.code == L.E_PATTERN


def test_configure_chunks_and_workspace_errors(L, box64):
    from paper_2104_08245_amd import Plan, NolsmError
    s = box64
    p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx)
    opts = L.default_opts("fp16")
    mb = p.configure(opts, 1 << 40)
    inf = p.info()
    # with room for everything, a chunk is cut only where the padded size
    # falls below 4/5 of the chunk's largest
    nps = sorted((((np.diff(s.K.row_ptr) * 6) + 63) // 64 * 64).tolist(), reverse=True)
    ranges, lead = 0, None
    for v in nps:
        if lead is None or 5 * v < 4 * lead:
            ranges, lead = ranges + 1, v
    assert inf["nchunks"] == ranges and mb == inf["meta_bytes"] > 0
    full = inf["ws_full_bytes"]
    p.configure(opts, full // 3)
    assert p.info()["nchunks"] >= 3
    with pytest.raises(NolsmError) as e:
        p.configure(opts, 1024)
    assert e.value.code == L.E_WORKSPACE
    opts.sched = L.SCHED_PER_BUCKET
    p.configure(opts, 1 << 40)
    m = np.diff(s.K.row_ptr) * 6
    buckets = len(set(((m + 63) // 64).tolist()))
    assert p.info()["nchunks"] == buckets


def test_bad_options_rejected(L, box64):
    from paper_2104_08245_amd import Plan, NolsmError
    s = box64
    p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx)
    for kw in (dict(prec=7), dict(max_iter=1), dict(max_iter=500), dict(sched=9), dict(inverse=5),
               dict(inverse=L.INV_COUPLED_NS),                       # FP64: 16-bit route only
               dict(inverse=L.INV_CHOLESKY_FP32),                    # FP64: 16-bit route only
               dict(inverse=L.INV_CHOLESKY_APPLY_FP32),              # FP64: 16-bit route only
               dict(inverse=4),
               dict(prec=L.PREC["fp32"], inverse=L.INV_CHOLESKY_FP32),
               dict(sym_sign=1),                                     # FP64: 16-bit only
               dict(prec=L.PREC["fp16"], sym_sign=1, inverse=L.INV_COUPLED_NS),
               dict(prec=L.PREC["fp16"], inverse=L.INV_COUPLED_NS, inv_max_iter=1)):
        opts = L.default_opts("fp64")
        for k, v in kw.items():
            setattr(opts, k, v)
        with pytest.raises(NolsmError) as e:
            p.configure(opts, 1 << 40)
        assert e.value.code == L.E_ARG


def _chain_pattern(nb):
    ptr, idx = [0], []
    for J in range(nb):
        idx.extend(I for I in (J - 1, J, J + 1) if 0 <= I < nb)
        ptr.append(len(idx))
    return np.array(ptr, np.int32), np.array(idx, np.int32)


def test_combination_equals_oracle(L, box64):
    # integer work: the library's groups must equal the oracle's exactly
    import synth
    from oracle import combine as cb
    from paper_2104_08245_amd import Plan
    cases = [("chain", 5, *_chain_pattern(5)), ("blockdiag", 8, np.arange(9, dtype=np.int32),
                                                  np.arange(8, dtype=np.int32))]
    slab = synth.water_slab(config_id=104, r_c=0.9, n_dense=96, n_dilute=96,
                            box=np.array([2.0, 2.0, 6.0]), z_split=1.4)
    for name, s in (("box64", box64), ("slab", slab)):
        cases.append((name, s.K.nb, s.K.row_ptr, s.K.col_idx))
    for name, nb, rp, ci in cases:
        p = Plan(nb, 6, rp, ci, flags=L.PLAN_COMBINE)
        got = p.groups()
        ex = p.export()
        want = cb.combine_groups(nb, ex["sub_ptr"], ex["sub_blk"])
        for a, b in zip(got, want):
            assert np.array_equal(a, b), name
        inf = p.info()
        assert inf["ngroups"] == len(want[0]) - 1
        assert inf["sum_gn3"] == cb.cubic_cost(want[0]) * 216.0
    # without the flag every molecule is its own submatrix
    p = Plan(box64.K.nb, 6, box64.K.row_ptr, box64.K.col_idx)
    g = p.groups()
    assert np.array_equal(g[2], np.arange(box64.K.nb + 1)) and np.array_equal(g[3], np.arange(box64.K.nb))


def test_default_route_is_fp64_cholesky_on_a(L):
    # every precision defaults to the FP64 factor and the sign of A_J itself
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        o = L.default_opts(prec)
        assert o.inverse == L.INV_CHOLESKY and o.sym_sign == 0


def test_pipeline_schedule_splits_the_workspace(L, box64):
    # two resident chunks: each gets half of the workspace
    from paper_2104_08245_amd import Plan, NolsmError
    s = box64
    p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx)
    g = L.default_opts("fp16")
    p.configure(g, 1 << 40)
    full = p.info()["ws_full_bytes"]
    for ws in (full, full // 2, full // 4):
        g = L.default_opts("fp16")
        p.configure(g, ws)
        n_graph = p.info()["nchunks"]
        o = L.default_opts("fp16", sched=L.SCHED_PIPELINE)
        p.configure(o, ws)
        assert p.info()["nchunks"] >= max(2, n_graph)
    # a workspace that holds the largest submatrix once, but not in each half,
    # serves the one-region schedules and is refused by the pipeline
    small = p.info()["ws_min_bytes"] + (1 << 20)
    p.configure(L.default_opts("fp16"), small)
    with pytest.raises(NolsmError) as e:
        p.configure(L.default_opts("fp16", sched=L.SCHED_PIPELINE), small)
    assert e.value.code == L.E_WORKSPACE


def test_switch_point_of_the_16bit_iteration(L):
    """The hand-over residual that nolsm_switch_tol returns, against what two
    (one) exact Newton-Schulz steps of the oracle (Eq. NS1) leave of it on a
    spectrum whose whole residual sits in one eigenvalue (the worst case:
    ||X^2 - I||_F bounds every |1 - x^2|): a tenth of the format's unit
    roundoff at leading order, the higher orders adding under 15%."""
    lib = L.lib()
    rng = np.random.default_rng(7)
    n = 96
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    signs = np.where(np.arange(n) % 3 == 0, -1.0, 1.0)
    for prec, u in (("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        for steps in (1, 2):
            r = lib.nolsm_switch_tol(L.PREC[prec], steps, -1.0)
            e = np.zeros(n)
            e[0] = r
            A = (Q * (signs * np.sqrt(1.0 - e))) @ Q.T
            assert abs(np.linalg.norm(A @ A - np.eye(n)) - r) < 1e-12
            X, _, _, _ = o.newton_schulz_sign(A, 1.0, tol=0.0, max_iter=steps)
            left = np.linalg.norm(X @ X - np.eye(n))
            assert u / 10 <= left <= 1.15 * u / 10, (prec, steps, r, left)
        assert lib.nolsm_switch_tol(L.PREC[prec], 0, -1.0) == 0.0
        assert lib.nolsm_switch_tol(L.PREC[prec], 2, 0.3) == 0.3
    assert lib.nolsm_switch_tol(L.PREC["fp64"], 0, -1.0) == 1e-10
    assert lib.nolsm_switch_tol(L.PREC["fp32"], 0, -1.0) == 1e-5
    # the defaults ask for the derived point in 16 bits only
    for prec in ("fp16", "bf16"):
        assert L.default_opts(prec).tol < 0
    assert L.default_opts("fp64").tol == 1e-10


def test_noalloc_refuses_plans_beyond_its_array(L, box64):
    # host-side checks of the allocation-free entry point, before any HIP call
    import ctypes as C
    from paper_2104_08245_amd import Plan
    s = box64
    p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx)
    opts = L.default_opts("fp16")
    p.configure(opts, 1 << 30)
    assert p.info()["ws_full_bytes"] > L.NOALLOC_WS_BYTES
    rc = L.lib().nolsm_sign_batch_noalloc(p.h, None, None, 0.0, C.byref(opts), None, None, None, None)
    assert rc == L.E_WORKSPACE
    assert b"scratch array" in L.lib().nolsm_strerror(rc)
    p.configure(opts, L.NOALLOC_WS_BYTES)
    assert p.info()["nchunks"] >= 2
    opts.sched = L.SCHED_PIPELINE
    rc = L.lib().nolsm_sign_batch_noalloc(p.h, None, None, 0.0, C.byref(opts), None, None, None, None)
    assert rc == L.E_ARG
    src = open(HEADER).read()
    m = re.search(r"#define NOLSM_NOALLOC_WS_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == L.NOALLOC_WS_BYTES


def test_largest_submatrix_limit(L):
    # full cells: every submatrix is the whole matrix, 6 rows per molecule;
    # 501 molecules give 3006 rows (accepted), 502 give 3012 (refused)
    import synth
    from paper_2104_08245_amd import Plan, NolsmError
    src = open(HEADER).read()
    m = re.search(r"#define NOLSM_MAX_ROWS (\d+)", src)
    assert m and int(m.group(1)) == L.MAX_ROWS
    for nmol, ok in ((501, True), (502, False)):
        s = synth.water_cube(nmol, 2.2, config_id=111)
        assert s.K.nnzb == nmol * nmol
        p = Plan(s.K.nb, s.K.bs, s.K.row_ptr, s.K.col_idx)
        opts = L.default_opts("fp16")
        if ok:
            p.configure(opts, 1 << 40)
            assert p.info()["m_max"] * 6 == 3006 <= L.MAX_ROWS
        else:
            with pytest.raises(NolsmError) as e:
                p.configure(opts, 1 << 40)
            assert e.value.code == L.E_ARG
