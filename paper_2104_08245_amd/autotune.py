"""Tile-shape autotuner for the FP16/BF16 Newton-Schulz GEMMs.

For every submatrix-size bucket (np = 64, 128, ... rows) present in a system,
times the Newton-Schulz phase with that bucket on 64x64 tiles and on 128x128
tiles (HIP events inside the library, `profile` option), keeps the faster
one, and returns the bitmask for `opts.ns_small_tile_mask`. Results are
cached as JSON keyed by (gfx950, precision, bucket).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib as L
from .nolsm import Solver

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_cache.json")


def buckets_of(system):
    m = np.diff(system.K.row_ptr)
    n = system.K.bs * m
    npd = (n + 63) // 64 * 64
    return sorted(set(int(x) for x in npd))


def ns_time(system, prec, mask, repeats=2, **kw):
    import torch
    sv = Solver(system, prec=prec, ns_small_tile_mask=mask, sched=L.SCHED_STREAM, **kw)
    best = None
    for _ in range(repeats):
        sv.set_opts(profile=1)
        sv.run()
        torch.cuda.synchronize()
        p = sv.profile()
        best = p["ms_ns"] if best is None else min(best, p["ms_ns"])
    return best


def tune(system, prec="fp16", log=print, cache=CACHE, **kw):
    """Greedy per bucket: flip the bucket's bit and keep the flip if the NS
    phase gets faster. Returns the mask."""
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    mask = L.default_opts(prec).ns_small_tile_mask
    base = ns_time(system, prec, mask, **kw)
    log(f"autotune {prec}: default mask {mask:#x}: NS {base:.2f} ms")
    for npd in buckets_of(system):
        bit = 1 << (npd // 64 - 1)
        trial = mask ^ bit
        t = ns_time(system, prec, trial, **kw)
        choice = 64 if (trial & bit) else 128
        if t < base:
            mask, base = trial, t
        else:
            choice = 64 if (mask & bit) else 128
        table[f"gfx950/{prec}/{npd}"] = choice
        log(f"  bucket np={npd}: {'64' if trial & bit else '128'}-row tiles {t:.2f} ms -> keep {choice}")
    if cache:
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return mask


def mask_from_cache(prec, cache=CACHE):
    """Mask from a cached table (buckets not in the table keep the default)."""
    mask = L.default_opts(prec).ns_small_tile_mask
    if not os.path.exists(cache):
        return mask
    with open(cache) as f:
        table = json.load(f)
    for key, tile in table.items():
        arch, p, npd = key.split("/")
        if arch != "gfx950" or p != prec:
            continue
        bit = 1 << (int(npd) // 64 - 1)
        mask = (mask | bit) if tile == 64 else (mask & ~bit)
    return mask
