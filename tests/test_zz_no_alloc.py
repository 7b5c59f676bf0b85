"""nolsm_sign_batch_noalloc (the library's static workspace array) against
nolsm_sign_batch with a caller workspace of the same size, through the C
ABI: two calls in a row on one GPU, the second on a smaller batch, so that
the second runs over the array as the first left it. Both entry points run
the same kernels over the same chunks, so the results agree bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def both(system, prec, **kw):
    import torch
    from paper_2104_08245_amd import Solver, _lib as L
    say(f"[gpu] noalloc vs workspace: nmol={system.nmol} prec={prec} {kw}")
    sv = Solver(system, prec=prec, device="cuda:0", ws_bytes=L.NOALLOC_WS_BYTES, sched=L.SCHED_STREAM, **kw)
    assert sv.plan.info()["nchunks"] >= 1
    sv.run()
    torch.cuda.synchronize()
    ref = (sv.Dcols.cpu().numpy().copy(), sv.D.cpu().numpy().copy(), sv.stats.cpu().numpy().copy())
    sv.Dcols.fill_(float("nan"))
    sv.D.fill_(float("nan"))
    sv.stats.fill_(0xFF)
    torch.cuda.synchronize()
    sv.run_noalloc()
    torch.cuda.synchronize()
    got = (sv.Dcols.cpu().numpy(), sv.D.cpu().numpy(), sv.stats.cpu().numpy())
    st = sv.host_stats()
    return sv, ref, got, st


def test_noalloc_matches_workspace_entry_point_twice(box64):
    import synth
    small = synth.water_cube(32, 0.55, config_id=1)
    for system, prec, kw in ((box64, "fp16", {"sym_sign": 1}), (small, "fp16", {"sym_sign": 1})):
        sv, ref, got, st = both(system, prec, **kw)
        say(f"  chunks {sv.plan.info()['nchunks']}, status ok {int((st['status'] == 0).sum())}/{system.nmol}")
        assert np.all(st["status"] == 0)
        for name, r, g in zip(("Dcols", "D", "stats"), ref, got):
            assert np.array_equal(r, g), name


def test_noalloc_fp64_after_fp16():
    import synth
    small = synth.water_cube(16, 0.5, config_id=1)
    sv, ref, got, st = both(small, "fp64")
    assert np.all(st["status"] == 0)
    for name, r, g in zip(("Dcols", "D", "stats"), ref, got):
        assert np.array_equal(r, g), name
