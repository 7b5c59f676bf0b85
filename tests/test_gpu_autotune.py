"""NS tile autotuner on the GPU: tuning writes a choice per size bucket, and
every tile choice (all 64x64, all 128x128, the tuned mix) gives the oracle's
result within the mixed-precision bounds, through the C ABI."""
import json
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
def ref1(box64):
    return o.nolsm(box64)


def check(sv, ref, prec, tag):
    st = sv.host_stats()
    assert np.all(st["status"] == 0)
    dc = sv.host_dcols()
    errs = np.array([np.linalg.norm(dc[J] - ref.Dcols[J]) / np.linalg.norm(ref.Dcols[J])
                     for J in range(len(ref.Dcols))])
    de = np.abs(st["energy_KD"] - ref.E)
    say(f"{tag}: Dcols rel-F max {errs.max():.3e}; |dE_J| max {de.max():.3e}")
    assert errs.max() <= MIXED[prec]["dcols"] and de.max() <= MIXED[prec]["energy"]
    return dc


@pytest.mark.parametrize("sym", [True, False])
def test_tuned_and_forced_tiles_match_oracle(box64, ref1, tmp_path, sym):
    import torch
    from paper_2104_08245_amd import Solver, autotune as at
    prec = "fp16"
    cache = str(tmp_path / "tiles.json")
    say(f"[gpu] autotune box64 {prec} sym={sym}")
    mask, choices = at.tune(box64, prec, sym, log=say, cache=cache, repeats=1)
    table = json.load(open(cache))
    assert set(table) == {at.key(prec, sym, b) for b in at.buckets_of(box64)} == set(choices)
    assert at.mask_for(box64, prec, sym, cache=cache)[0] == mask
    every = sum(at.bit_of(b) for b in at.buckets_of(box64))
    sv = Solver(box64, prec=prec, device="cuda:0", sym_sign=int(sym), ns_small_tile_mask=mask)
    results = {}
    for tag, m in (("tuned", mask), ("all 64", every), ("all 128", 0)):
        say(f"[gpu] tiles {tag} mask {m:#x}")
        sv.reconfigure(ns_small_tile_mask=m)
        sv.run()
        torch.cuda.synchronize()
        results[tag] = check(sv, ref1, prec, f"{prec} sym={sym} {tag}")
    # reconfiguring back reproduces the first run bit for bit
    sv.reconfigure(ns_small_tile_mask=mask)
    sv.run()
    torch.cuda.synchronize()
    assert all(np.array_equal(a, b) for a, b in zip(sv.host_dcols(), results["tuned"]))
