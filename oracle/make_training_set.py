"""Writes the learned-bounds training set: features and eigensolve labels of
submatrices A_J = S_J^-1 K_J - mu I drawn from fresh instances of the
homogeneous (4096 and 32768 molecules, r_c 0.9 nm) and slab (16384
molecules, r_c 1.2 nm) generators, with seeds different from every
evaluation system. Calls only the oracle and the input generator.

TEST INFRASTRUCTURE (oracle side): run as
    python -m oracle.make_training_set [N] [out.npz] [processes]
or, for the features of the symmetric similar matrix L^-1 K_J L^-T - mu I
of the same submatrices (labels copied):
    python -m oracle.make_training_set --sym [processes]
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import mlp  # noqa: E402
from oracle import nolsm as o  # noqa: E402

# (generator, config seed id, share of the set)
SOURCES = [("cube4096", 1002, 0.2), ("cube4096", 2002, 0.2), ("cube32768", 1003, 0.4),
           ("slab16384", 1004, 0.2)]

_SYS = None


def _single_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def make(kind, cid):
    if kind == "cube4096":
        return synth.water_cube(4096, 0.9, config_id=cid)
    if kind == "cube32768":
        return synth.water_cube(32768, 0.9, config_id=cid)
    return synth.water_slab(config_id=cid, r_c=1.2)


def one(J):
    s = _SYS
    lists, self_pos = o.neighbour_lists(s)
    idx = lists[J]
    KJ = o.gather_vectorized(idx, 6, s.K.row_ptr, s.K.col_idx, s.K.val)
    SJ = o.gather_vectorized(idx, 6, s.S.row_ptr, s.S.col_idx, s.S.val)
    A = np.linalg.solve(SJ, KJ) - s.mu * np.eye(KJ.shape[0])
    f = mlp.features(A)
    lo, hi = mlp.labels(KJ, SJ, s.mu)
    return J, f, lo, hi, KJ.shape[0]


def one_sym(J):
    # the same submatrix, features of A~ = L^-1 K_J L^-T - mu I instead of A_J
    s = _SYS
    lists, self_pos = o.neighbour_lists(s)
    idx = lists[J]
    KJ = o.gather_vectorized(idx, 6, s.K.row_ptr, s.K.col_idx, s.K.val)
    SJ = o.gather_vectorized(idx, 6, s.S.row_ptr, s.S.col_idx, s.S.val)
    return J, mlp.features_symmetric(KJ, SJ, s.mu), KJ.shape[0]


def main_sym(src=None, out=None, procs=None):
    """Features of A~ for exactly the submatrices of the A_J set (same
    generators, seeds and draws, same order); the labels (extreme eigenvalues
    of the pencil, shared by A_J and A~) are copied from that set."""
    global _SYS
    src = src or os.path.join(ROOT, "tests", "golden", "mlp_train.npz")
    out = out or os.path.join(ROOT, "tests", "golden", "mlp_train_sym.npz")
    procs = procs or min(8, os.cpu_count() or 1)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    base = np.load(src)
    total = len(base["labels"])
    F, N = [], []
    for si, (kind, cid, share) in enumerate(SOURCES):
        t = time.time()
        s = make(kind, cid)
        o.neighbour_lists(s)
        _SYS = s
        rng = np.random.default_rng(cid)
        cnt = min(int(round(total * share)), s.nmol)
        Js = sorted(rng.choice(s.nmol, cnt, replace=False).tolist())
        with mp.get_context("fork").Pool(procs, initializer=_single_thread) as pool:
            res = pool.map(one_sym, Js, chunksize=8)
        for J, f, n in res:
            F.append(f)
            N.append(n)
        print(f"{kind} seed {cid}: {cnt} submatrices in {time.time() - t:.0f}s", flush=True)
    N = np.array(N, np.int32)
    if not np.array_equal(N, base["n"]):
        raise RuntimeError("regenerated submatrices differ from the A_J set")
    np.savez_compressed(out, features=np.array(F, np.float64), labels=base["labels"], n=N,
                        source=base["source"])
    print("wrote", out, len(F))


def main(total=20000, out=None, procs=None):
    global _SYS
    out = out or os.path.join(ROOT, "tests", "golden", "mlp_train.npz")
    procs = procs or min(8, os.cpu_count() or 1)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    F, Y, N, SRC = [], [], [], []
    for si, (kind, cid, share) in enumerate(SOURCES):
        t = time.time()
        s = make(kind, cid)
        o.neighbour_lists(s)
        _SYS = s
        rng = np.random.default_rng(cid)
        cnt = min(int(round(total * share)), s.nmol)
        Js = sorted(rng.choice(s.nmol, cnt, replace=False).tolist())
        with mp.get_context("fork").Pool(procs, initializer=_single_thread) as pool:
            res = pool.map(one, Js, chunksize=8)
        for J, f, lo, hi, n in res:
            F.append(f)
            Y.append((lo, hi))
            N.append(n)
            SRC.append(si)
        print(f"{kind} seed {cid}: {cnt} submatrices in {time.time() - t:.0f}s", flush=True)
    np.savez_compressed(out, features=np.array(F, np.float64), labels=np.array(Y, np.float64),
                        n=np.array(N, np.int32), source=np.array(SRC, np.int8))
    print("wrote", out, len(F))


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "--sym":
        main_sym(procs=int(a[1]) if len(a) > 1 else None)
    else:
        main(int(a[0]) if a else 20000, a[1] if len(a) > 1 else None, int(a[2]) if len(a) > 2 else None)
