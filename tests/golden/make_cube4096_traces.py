"""Writes tests/golden/cube4096_traces.npz: the FP64 oracle's per-molecule
traces N_J = sum_c (S_J Dcols_J)[cJ_c, c] and band energies
E_J = sum_c (K_J Dcols_J)[cJ_c, c] (Sec. III-B.2, owned columns of
Eq. purification_submatrix) for every molecule of the 4,096-molecule
water-like cube at r_c 0.9 nm and mu = 0, with a digest of the generated K
and S values so that a test can tell that it compares the same system.
Calls only the input generator and the oracle.

TEST INFRASTRUCTURE (oracle side): run as
    python tests/golden/make_cube4096_traces.py [processes]
"""
from __future__ import annotations

import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import nolsm as o  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube4096_traces.npz")
_SYS = None


def system_digest(s):
    h = hashlib.sha256()
    for a in (s.K.row_ptr, s.K.col_idx, s.K.val, s.S.row_ptr, s.S.col_idx, s.S.val):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _single_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _one(J):
    r = o.solve_molecule(_SYS, J)
    return J, r.status, r.N_J, r.E_J, r.iters


def main():
    global _SYS
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    _SYS = synth.make_config(2)
    o.neighbour_lists(_SYS)
    nmol = _SYS.nmol
    t = time.time()
    with mp.get_context("fork").Pool(procs, initializer=_single_thread) as pool:
        res = pool.map(_one, range(nmol), chunksize=8)
    N = np.zeros(nmol)
    E = np.zeros(nmol)
    status = np.zeros(nmol, np.int32)
    iters = np.zeros(nmol, np.int32)
    for J, st, n, e, it in res:
        N[J], E[J], status[J], iters[J] = n, e, st, it
    np.savez(OUT, N=N, E=E, status=status, iters=iters, digest=np.array(system_digest(_SYS)))
    print(f"{nmol} molecules in {time.time() - t:.0f}s with {procs} processes; "
          f"N_J {N.min():.4f}..{N.max():.4f}, all OK: {bool(np.all(status == 0))} -> {OUT}")


if __name__ == "__main__":
    main()
