"""Tile-shape autotuner for the FP16/BF16 Newton-Schulz products.

For every submatrix-size bucket (np = 64, 128, ... rows) of a system, times
the Newton-Schulz phase (HIP events inside the library, `profile` option)
with that bucket on 64x64 tiles and on 128x128 tiles, keeps the faster one,
and returns the bitmask for `opts.ns_small_tile_mask`. The choices are
cached as JSON keyed by architecture, precision, iteration variant
(symmetric, or on A_J) and bucket; `mask_for` turns the cache into the mask
for another system, and says which of its buckets the cache covered.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib as L

ARCH = "gfx950"
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_cache.json")


def key(prec, sym, npd):
    return f"{ARCH}/{prec}/{'sym' if sym else 'plain'}/{int(npd)}"


def bit_of(npd):
    return 1 << (int(npd) // 64 - 1)


def buckets_of(system):
    """Padded sizes np (multiples of 64) of the system's submatrices, one
    per molecule (the plan's buckets when submatrices are not combined)."""
    m = np.diff(system.K.row_ptr)
    npd = (system.K.bs * m + 63) // 64 * 64
    return sorted(set(int(x) for x in npd))


def load_table(cache=CACHE):
    if cache and os.path.exists(cache):
        with open(cache) as f:
            return json.load(f)
    return {}


def mask_for(system, prec, sym, cache=CACHE, table=None):
    """(mask, tuned, buckets): the default mask with every bucket of the
    system that the cache holds set to its tuned tile; `tuned` lists those
    buckets."""
    table = load_table(cache) if table is None else table
    mask = L.default_opts(prec).ns_small_tile_mask
    buckets = buckets_of(system)
    tuned = []
    for npd in buckets:
        tile = table.get(key(prec, sym, npd))
        if tile is None:
            continue
        if tile not in (64, 128):
            raise ValueError(f"tile cache: {key(prec, sym, npd)} -> {tile}")
        mask = (mask | bit_of(npd)) if tile == 64 else (mask & ~bit_of(npd))
        tuned.append(npd)
    return mask, tuned, buckets


def ns_time(sv, mask, repeats):
    """Shortest NS phase over `repeats` solves with the given tile mask."""
    import torch
    sv.reconfigure(ns_small_tile_mask=mask)
    best = None
    for _ in range(repeats):
        sv.set_opts(profile=1)
        sv.run()
        torch.cuda.synchronize()
        t = sv.profile()["ms_ns"]
        best = t if best is None else min(best, t)
    sv.set_opts(profile=0)
    return best


def tune(system, prec="fp16", sym=True, log=print, cache=CACHE, repeats=3, **solver_kw):
    """Greedy per bucket, largest first: flip the bucket's bit and keep the
    flip if the NS phase gets faster. Merges the choices into `cache` (if
    given) and returns (mask, {key: tile})."""
    from .nolsm import Solver
    if prec not in ("fp16", "bf16"):
        raise ValueError("the tile choice exists for the 16-bit iteration only")
    sv = Solver(system, prec=prec, sched=L.SCHED_STREAM, sym_sign=int(sym), **solver_kw)
    mask = L.default_opts(prec).ns_small_tile_mask
    base = ns_time(sv, mask, repeats)
    log(f"autotune {prec} {'sym' if sym else 'plain'}: default mask {mask:#x}: NS {base:.2f} ms")
    choices = {}
    for npd in sorted(buckets_of(system), reverse=True):
        b = bit_of(npd)
        trial = mask ^ b
        t = ns_time(sv, trial, repeats)
        if t < base:
            mask, base = trial, t
        choices[key(prec, sym, npd)] = 64 if mask & b else 128
        log(f"  np={npd}: {64 if trial & b else 128}-row tiles {t:.2f} ms -> keep "
            f"{choices[key(prec, sym, npd)]}")
    if cache:
        table = load_table(cache)
        table.update(choices)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
            f.write("\n")
    del sv
    return mask, choices
