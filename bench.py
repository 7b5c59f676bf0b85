#!/usr/bin/env python3
"""Benchmark of the batched NOLSM sign solve on one MI355X.

One step = one nolsm_sign_batch call over the whole synthetic system: gather
-> FP64 Cholesky/substitution -> bounds -> Newton-Schulz (FP16/BF16 MFMA with
FP32 accumulation, or FP32/FP64) -> FP32 finishing iterations -> extraction,
traces and write-back into the block-sparse D. Inputs are resident in HBM
before the timed region; the graph-captured batch is replayed K times.

metric: TFLOP/s of the Newton-Schulz GEMMs as executed on the true
submatrix size (2 n^3 per n x n product on A_J; n^2 (n + 1) per product of
the symmetric iteration, which forms the unique half of each symmetric
product), plus the finishing products at their algorithmic 12 n^2 per n x 6
product, divided by the end-to-end step time; submatrices/s beside it. The
paper's count (2 n^3 per product of the sign iteration, Sec. IV-B) is
reported under its own key.

Prints one JSON line. Also measures, outside the timed region: the phase
times of one profiled step (HIP events) for the roofline of the dominant
kernel; timed legs of the iteration on A_J = S^-1 K - mu I (no symmetric
form) and of the plain FP64 GPU path on the same batch; the per-molecule
band-energy error of a sample against the FP64 CPU oracle; the density-matrix
checks of the assembled D against the FP64 GPU solve; and the oracle's own
throughput on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
WORKLOAD = {1: "water-like cube, 64 molecules, r_c 0.6 nm",
            2: "water-like cube, 4096 molecules, r_c 0.9 nm",
            3: "water-like cube, 32768 molecules, r_c 0.9 nm",
            4: "water-like two-density slab, 16384 molecules, r_c 1.2 nm"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_ns_lp_fp16_cube32768_traffic.md")
# the sign-iteration kernel and its shared tile loop
NS_SOURCES = [os.path.join(ROOT, "paper_2104_08245_amd", "csrc", f) for f in ("k_ns.hip", "lp_gemm.h")]


def measured_traffic(config, prec, sym, mean_iters, combine):
    """HBM bytes per NS launch from the committed FETCH_SIZE/WRITE_SIZE
    summary (copy-calibrated), or None when the summary does not cover this
    workload and kernel variant (one submatrix per molecule), the kernel
    source has changed since the counters were taken, or the iterations per
    submatrix differ (the average runs over every launch of a step,
    converged ones included)."""
    import hashlib
    if config != 3 or prec != "fp16" or combine or not os.path.exists(TRAFFIC_FILE):
        return None
    sha, nbytes, variant, iters = None, None, None, None
    for line in open(TRAFFIC_FILE):
        if line.startswith("kernel_sources_sha256 "):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("k_ns_lp variant:"):
            variant = line.split(":", 1)[1].strip()
        elif line.startswith("k_ns_lp traffic_bytes_per_launch:"):
            nbytes = int(line.split(":", 1)[1])
        elif line.startswith("k_ns_lp mean_iterations:"):
            iters = float(line.split(":", 1)[1])
    h = hashlib.sha256()
    for f in NS_SOURCES:
        h.update(open(f, "rb").read())
    cur = h.hexdigest()
    ok = (sha == cur and nbytes and variant == ("sym" if sym else "plain") and iters is not None
          and abs(iters - mean_iters) <= 0.05)
    return nbytes if ok else None


# ------------------------------------------------------- density-matrix checks
DENSITY_PROBES = 16


def density_against_fp64(system, ex, Dm_host, ref):
    """Idempotency ||D S D - D||_F / ||D||_F (probe estimate), asymmetry and
    Tr(D S) per molecule of the assembled D of the timed solve (Dm_host) and
    of the FP64 solve of the same batch on the GPU (`ref`, whose D equals
    the FP64 oracle's to 1e-10 in the parity tests; the oracle itself would
    take hours here), with the relative Frobenius difference of the two D."""
    import scipy.sparse.linalg as spla
    from paper_2104_08245_amd import diagnostics as dg
    t0 = time.time()
    nb, bs = system.K.nb, system.K.bs
    S = dg.block_csr(nb, bs, system.S.row_ptr, system.S.col_idx, system.S.val)
    Dm = dg.block_csr(nb, bs, ex["D_row_ptr"], ex["D_col_idx"], Dm_host)
    res = {"probes": DENSITY_PROBES,
           "mixed": dg.density_checks(Dm, S, system.nmol, probes=DENSITY_PROBES, seed=11)}
    D64 = dg.block_csr(nb, bs, ex["D_row_ptr"], ex["D_col_idx"], ref.host_D())
    res["fp64_gpu"] = dg.density_checks(D64, S, system.nmol, probes=DENSITY_PROBES, seed=11)
    res["rel_diff_D_vs_fp64"] = float(spla.norm(Dm - D64) / spla.norm(D64))
    log(f"density checks: {time.time() - t0:.1f}s")
    return res


def paper_and_exec_flops(sv, sym, system):
    """Per solved submatrix (one per molecule, or one per group when
    combined): its rows n and the iteration counts of its first owned
    molecule; returns the flop counts of the sign iteration (the paper's
    2 n^3 per product, and what executes: n^2 (n + 1) per product of the
    symmetric form), of the finishing products, and the arrays behind them."""
    import numpy as np
    st = sv.host_stats()
    grp_ptr, _, own_ptr, own_J = sv.plan.groups()
    n = sv.bs * np.diff(grp_ptr).astype(np.float64)
    first = own_J[own_ptr[:-1]]
    ok = np.array([np.all(st["status"][own_J[own_ptr[g]:own_ptr[g + 1]]] == 0) for g in range(len(n))])
    it = st["iters"][first].astype(np.float64)
    paper = float(((2 * it + 1) * 2.0 * n ** 3)[ok].sum())
    execd = float(((2 * it + 1) * n ** 2 * (n + 1))[ok].sum()) if sym else paper
    nfin = st["iters_fp32"][first].astype(np.float64)
    nown = np.diff(own_ptr).astype(np.float64)
    fin = float((nown * np.where(nfin == 2, 9, np.where(nfin == 1, 3, 1)) * 12.0 * n ** 2)[ok].sum())
    return dict(paper=paper, exec=execd, fin=fin, n=n, it=it, ok=ok, first=first, nown=nown, st=st)


def time_leg(system, dev, args, label, steps, **kw):
    """A solver of the same batch with other options, warmed once and timed
    over `steps` steps on its own stream (the graph schedule)."""
    import torch
    from paper_2104_08245_amd import Solver
    sv = Solver(system, device=dev, ws_budget=int(args.ws_gb * (1 << 30)), combine=args.combine, **kw)
    stream = torch.cuda.Stream(device=dev)
    sv.run(stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        sv.run(stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / steps
    log(f"leg {label}: {steps} steps, {ms:.1f} ms/step")
    return sv, ms


# ------------------------------------------------------------------ CPU leg
_SYS = None


def _single_thread():
    # numpy's BLAS pool was created before the fork: limit it in each worker
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _oracle_one(J):
    from oracle import nolsm as o
    t = time.perf_counter()
    r = o.solve_molecule(_SYS, J)
    dt = time.perf_counter() - t
    n = r.Dcols.shape[0]
    return J, r.E_J, r.iters, n, dt


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, sample, workers, single):
    """The FP64 oracle on `sample` molecules, one process per core (BLAS
    single-threaded), forked before any GPU use; and on the first `single`
    of them in this process alone, single-threaded (the one-core rate)."""
    global _SYS
    from threadpoolctl import threadpool_limits
    from oracle import nolsm as o
    _SYS = system
    o.neighbour_lists(system)
    with threadpool_limits(1):
        t = time.perf_counter()
        one = [_oracle_one(J) for J in sample[:single]]
        wall1 = time.perf_counter() - t
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(workers, initializer=_single_thread) as pool:
        res = pool.map(_oracle_one, sample, chunksize=1)
    wall = time.perf_counter() - t
    fl = lambda rs: sum((2 * it + 1) * 2.0 * n ** 3 for _, _, it, n, _ in rs)
    return dict(wall=wall, flops=fl(res), E={J: e for J, e, _, _, _ in res}, n=len(res),
                single=dict(n=len(one), wall=wall1, flops=fl(one)))


def bounds_eval(args):
    """Learned vs Gershgorin spectral bounds on the trajectory workload: the
    MLP is trained with the library's kernels on the oracle-labelled set in
    tests/golden, then every frame is solved in FP16 with both bounds. The
    energy error of each is taken against the FP64 GPU solve of the same
    frame (which matches the oracle to 1e-10 relative)."""
    import numpy as np
    import torch
    import synth
    from paper_2104_08245_amd import Solver, _lib as L
    from paper_2104_08245_amd import learned

    dev = torch.device("cuda:0")
    # the default path iterates on L^-1 K L^-T - mu I (FP64 factor applied in
    # FP32): its network is trained on that matrix's features; --no-sym
    # evaluates the iteration on A_J with the network of A_J's features
    sym = args.sym
    path = dict(sym_sign=1, inverse=L.INV_CHOLESKY_APPLY_FP32) if sym else {}
    ts = np.load(os.path.join(ROOT, "tests", "golden", "mlp_train_sym.npz" if sym else "mlp_train.npz"))
    t0 = time.perf_counter()
    tr = learned.train(ts["features"], ts["labels"], epochs=200, device=dev)
    torch.cuda.synchronize()
    log(f"trained the MLP on {len(ts['labels'])} submatrices in {time.perf_counter() - t0:.1f}s")
    frames = synth.trajectory(nframes=10)
    log(f"generated {len(frames)} frames of {frames[0].nmol} molecules")
    res = {"gershgorin": [[], 0, []], "learned": [[], 0, []]}
    ms = {"gershgorin": 0.0, "learned": 0.0}
    for f, sysf in enumerate(frames):
        ref = Solver(sysf, prec="fp64", device=dev)
        ref.run()
        torch.cuda.synchronize()
        e64 = ref.host_stats()["energy_KD"]
        del ref
        for mode in ("gershgorin", "learned"):
            kw = {}
            if mode == "learned":
                kw = dict(bounds=L.BOUNDS_LEARNED, d_mlp=tr["params"].data_ptr(),
                          d_mlp_norm=tr["norm"].data_ptr())
            sv = Solver(sysf, prec="fp16", device=dev, **path, **kw)
            sv.run()
            torch.cuda.synchronize()
            t = time.perf_counter()
            sv.run()
            torch.cuda.synchronize()
            ms[mode] += 1e3 * (time.perf_counter() - t)
            st = sv.host_stats()
            res[mode][0].append(st["iters"].astype(np.int64))
            res[mode][1] += int(st["fallback"].sum())
            res[mode][2].append(np.abs(st["energy_KD"] - e64))
            del sv
        log(f"frame {f}: gershgorin {res['gershgorin'][0][-1].mean():.3f}, "
            f"learned {res['learned'][0][-1].mean():.3f} mean iterations")
    out = {"metric": "NS iterations per submatrix, learned vs Gershgorin bounds",
           "data": "synthetic", "dtype": "f16",
           "config": {"workload": "10-frame water-like trajectory, 4096 molecules, r_c 0.9 nm",
                      "frames": len(frames), "molecules": frames[0].nmol,
                      "iteration_on": "L^-1 K L^-T - mu I (FP64 factor applied in FP32)" if sym
                      else "A = S^-1 K - mu I"}}
    for mode, (its, fb, dE) in res.items():
        its = np.concatenate(its)
        dE = np.concatenate(dE)
        vals, cnt = np.unique(its, return_counts=True)
        out[mode] = {"mean_iters": round(float(its.mean()), 4),
                     "histogram": {int(v): int(c) for v, c in zip(vals, cnt)},
                     "restarts": fb, "ms_per_frame": round(ms[mode] / len(frames), 2),
                     "energy_error_vs_fp64_gpu": {"max": float(dE.max()), "mean": float(dE.mean())}}
    g, l = out["gershgorin"]["mean_iters"], out["learned"]["mean_iters"]
    out["iterations_saved_per_submatrix"] = round(g - l, 4)
    out["iterations_saved_frac"] = round((g - l) / g, 4)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--prec", default="fp16", choices=list(PEAK_TFLOPS))
    ap.add_argument("--ws-gb", type=float, default=160.0)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sched", default="graph", choices=["graph", "stream", "bucket", "persistent", "pipeline"])
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB "
                         "(reference for the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--inverse", default="auto",
                    choices=["auto", "cholesky", "cholesky_apply_fp32", "cholesky_fp32", "coupled_ns"],
                    help="route to T_J(S)^-1: FP64 Cholesky (the default of FP64/FP32), FP64 Cholesky "
                         "applied through its FP32 copy with FP32 arithmetic (16-bit only; their "
                         "default), Cholesky and substitution both in FP32 (16-bit only), or the "
                         "coupled Newton-Schulz iteration in the NS precision (16-bit only)")
    ap.add_argument("--want-w", action="store_true",
                    help="also compute the energy-weighted density matrix columns each step")
    ap.add_argument("--sym", action=argparse.BooleanOptionalAction, default=True,
                    help="run the 16-bit sign iteration on the symmetric similar matrix "
                         "L^-1 K L^-T - mu I (upper GEMM tiles only, mirrored; default on, "
                         "--no-sym iterates on A = S^-1 K - mu I)")
    ap.add_argument("--density", action=argparse.BooleanOptionalAction, default=True,
                    help="16-bit runs: idempotency, asymmetry and trace of the assembled D, and of the "
                         "FP64 GPU solve of the same batch (after the timed steps)")
    ap.add_argument("--finish-rows", action="store_true",
                    help="FP16: the finishing products with the row-streaming vector kernel (one "
                         "launch per product) instead of the fused matrix-core kernel")
    ap.add_argument("--subst-fp32", action="store_true",
                    help="symmetric route with FP32 substitutions: their tile products on the FP32 "
                         "matrix cores instead of the default split FP16 (hi/lo) products")
    ap.add_argument("--tiles", default="cache", choices=["cache", "tune", "default"],
                    help="16-bit NS tile per size bucket: the autotuned choices of the tile cache "
                         "(buckets it lacks keep the default), tune them now before the warm-up "
                         "(untimed; written to --tile-cache), or the library's default mask")
    ap.add_argument("--tile-cache", default=None,
                    help="tile cache JSON (default: the package's tile_cache.json)")
    ap.add_argument("--combine", action="store_true",
                    help="combine submatrices (cubic criterion) before solving")
    ap.add_argument("--legs", action=argparse.BooleanOptionalAction, default=True,
                    help="16-bit runs: also time, after the main steps, the iteration on "
                         "A = S^-1 K - mu I (when the main line is symmetric) and the plain FP64 "
                         "GPU path on the same batch")
    ap.add_argument("--leg-steps", type=int, default=3, help="timed steps of the 16-bit leg")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed steps of the FP64 leg")
    ap.add_argument("--bounds-eval", action="store_true",
                    help="instead of the throughput line: NS iteration counts with learned vs "
                         "Gershgorin bounds over the 10-frame trajectory (FP16)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(every submatrix is independent, so molecules would be split across GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synth

    if args.bounds_eval:
        bounds_eval(args)
        return

    t0 = time.perf_counter()
    system = synth.make_config(args.config)
    log(f"generated config {args.config}: {system.nmol} molecules, nnzb {system.K.nnzb} "
        f"({time.perf_counter() - t0:.1f}s)")
    rng = np.random.default_rng(12345)

    cpu = None
    if not args.no_cpu:
        # one process per host core of this job's share: the GPU machine gives one
        # GPU's job 16 of its cores, whatever the machine's total
        share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        workers = args.cpu_workers or min(16, share)
        # about 10-20 s of oracle work on the cores of this job: 40 molecules
        # per process (0.25-0.5 s each at these sizes)
        nsample = args.cpu_sample or 40 * workers
        sample = sorted(rng.choice(system.nmol, size=min(nsample, system.nmol), replace=False).tolist())
        log(f"cpu baseline: oracle on {len(sample)} molecules with {workers} processes")
        cpu = cpu_baseline(system, sample, workers, single=min(4, len(sample)))
        cpu.update(workers=workers, share=share)
        log(f"cpu baseline: {cpu['wall']:.1f}s ({cpu['single']['wall']:.1f}s on one core)")

    import torch
    from paper_2104_08245_amd import Solver, _lib as L

    sched = {"graph": L.SCHED_GRAPH, "stream": L.SCHED_STREAM, "bucket": L.SCHED_PER_BUCKET,
             "persistent": L.SCHED_PERSISTENT, "pipeline": L.SCHED_PIPELINE}[args.sched]
    dev = torch.device("cuda:0")
    if args.inverse == "auto":
        args.inverse = "cholesky_apply_fp32" if args.prec in ("fp16", "bf16") else "cholesky"
    inv = {"cholesky": L.INV_CHOLESKY, "cholesky_apply_fp32": L.INV_CHOLESKY_APPLY_FP32,
           "cholesky_fp32": L.INV_CHOLESKY_FP32, "coupled_ns": L.INV_COUPLED_NS}[args.inverse]
    sym = 1 if (args.sym and args.prec in ("fp16", "bf16") and args.inverse != "coupled_ns"
                and not args.want_w) else 0
    lowp = args.prec in ("fp16", "bf16")
    tiles, masks = None, {}
    if lowp:
        from paper_2104_08245_amd import autotune
        cache = args.tile_cache or autotune.CACHE
        if args.tiles == "tune":
            autotune.tune(system, args.prec, bool(sym), log=log, cache=cache, inverse=inv,
                          combine=args.combine, ws_budget=int(args.ws_gb * (1 << 30)))
            torch.cuda.empty_cache()
        for v in (True, False):
            if args.tiles == "default":
                masks[v] = (L.default_opts(args.prec).ns_small_tile_mask, [], autotune.buckets_of(system))
            else:
                masks[v] = autotune.mask_for(system, args.prec, v, cache=cache)
        mask, tuned, buckets = masks[bool(sym)]
        tiles = {"mask": hex(mask), "source": "library default" if args.tiles == "default" else
                 "autotuned" if args.tiles == "tune" else "tile cache",
                 "buckets_tuned": f"{len(tuned)}/{len(buckets)}"}
        log(f"NS tiles: mask {mask:#x}, {tiles['source']}, {tiles['buckets_tuned']} buckets tuned")
    tile_kw = {"ns_small_tile_mask": masks[bool(sym)][0]} if lowp else {}
    sv = Solver(system, prec=args.prec, device=dev, ws_budget=int(args.ws_gb * (1 << 30)), sched=sched,
                inverse=inv, combine=args.combine, sym_sign=sym, finish_rows=1 if args.finish_rows else 0,
                subst_fp32=1 if args.subst_fp32 else 0, **tile_kw)
    if args.want_w:
        sv.want_w()
    info = sv.plan.info()
    log(f"plan: {info['nchunks']} chunks, {info['ngroups']} submatrices, "
        f"workspace {sv.ws_bytes / 2**30:.1f} GiB")
    stream = torch.cuda.Stream(device=dev)
    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calib_mib} MiB read + written")
        del src, dst
    for w in range(args.warmup):
        sv.run(stream=stream)
        stream.synchronize()
        log(f"warmup {w} done")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(args.steps):
        sv.run(stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms = 1e3 * elapsed / args.steps
    log(f"timed {args.steps} steps: {ms:.1f} ms/step")

    fl = paper_and_exec_flops(sv, sym, system)
    st, n, it, ok, first, nown = fl["st"], fl["n"], fl["it"], fl["ok"], fl["first"], fl["nown"]
    gemm_flops, exec_gemm_flops, fin_flops = fl["paper"], fl["exec"], fl["fin"]
    # coupled Newton-Schulz inverse: K+1 residual GEMMs, 2K updates, Z^2 and
    # S^-1 K, each 2 n^3 like every counted GEMM
    iti = st["iters_inv"][first].astype(np.float64)
    inv_flops = float(((3 * iti + 3) * 2.0 * n ** 3)[ok].sum()) if args.inverse == "coupled_ns" else 0.0
    tflops = (exec_gemm_flops + inv_flops + fin_flops) / (ms / 1e3) / 1e12
    tflops_paper = (gemm_flops + inv_flops + fin_flops) / (ms / 1e3) / 1e12

    # one profiled step (direct launches, HIP events between phases)
    sv.set_opts(profile=1)
    sv.run(stream=stream)
    prof = sv.profile()
    sv.set_opts(profile=0)
    ns_tf = exec_gemm_flops / (prof["ms_ns"] / 1e3) / 1e12 if prof["ms_ns"] > 0 else 0.0
    peak = PEAK_TFLOPS[args.prec]
    roofline = {"bound": "mfma", "achieved": round(ns_tf, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ns_tf / peak, 4), "traffic": measured_traffic(args.config, args.prec, sym, float(it.mean()),
                                                                    args.combine),
                "kernel": (("k_ns_lp" + ("<sym>" if sym else "")) + " (k_ns_lp_tail from iteration 16)")
                if args.prec in ("fp16", "bf16") else "k_ns64",
                "launches": prof["n_ns_launches"],
                "avg_launch_ms": round(prof["ms_ns"] / max(1, prof["n_ns_launches"]), 4)}
    phases = {k: round(v, 2) for k, v in prof.items()
              if k.startswith("ms_") and (k != "ms_wmat" or args.want_w)
              and (k != "ms_inverse" or args.inverse == "coupled_ns")
              and (k not in ("ms_chol", "ms_subst") or args.inverse != "coupled_ns")}
    # composite bound: each phase's algorithmic work at its own peak (NS GEMMs
    # on the MFMA peak of the precision, finishing products at the FP32 peak,
    # the Cholesky + solves at the FP64 or FP32 peak of their route, FP32
    # solves formed as split FP16 products (symmetric route) at a third of the
    # FP16 peak, the gather at 8 TB/s)
    m = n / 6.0
    setup_flops = float((n ** 3 / 3.0 + 2.0 * n ** 3 + 12.0 * n ** 2).sum())
    gather_bytes = float((576.0 * m ** 2 + 288.0 * m).sum())
    terms = {"ns": exec_gemm_flops / (peak * 1e12), "finish": fin_flops / 157.3e12,
             "gather_scatter": gather_bytes / 8e12}
    if args.inverse == "coupled_ns":
        terms["inverse"] = inv_flops / (peak * 1e12)
    elif args.inverse in ("cholesky_fp32", "cholesky_apply_fp32"):
        chol_flops = float((n ** 3 / 3.0).sum())
        split = bool(sym) and not args.subst_fp32
        apply_peak = 2500e12 / 3.0 if split else 157.3e12
        if args.inverse == "cholesky_fp32":
            terms["setup_fp32_factor"] = chol_flops / 157.3e12
        else:
            terms["setup_fp64_factor"] = chol_flops / 78.6e12
        terms["setup_fp32_apply_split16" if split else "setup_fp32_apply"] = (setup_flops - chol_flops) / apply_peak
    else:
        terms["setup_fp64"] = setup_flops / 78.6e12
    t_bound = sum(terms.values())
    composite = {"ms": round(1e3 * t_bound, 2), "frac": round(1e3 * t_bound / ms, 4),
                 "terms_ms": {k: round(1e3 * v, 2) for k, v in terms.items()}}

    out = {
        "metric": "NOLSM sign-solve TFLOP/s + submatrices/s, mixed vs FP64 at stated energy error",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp16": "f16", "bf16": "bf16", "fp32": "f32", "fp64": "f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": WORKLOAD.get(args.config, str(args.config)), "molecules": system.nmol,
                   "submatrix_rows": [int(n.min()), int(round(n.mean())), int(n.max())],
                   "precision": args.prec, "schedule": args.sched, "inverse": args.inverse,
                   "combined": bool(args.combine), "symmetric_sign": bool(sym), "submatrices": int(len(n)),
                   "finishing": "row kernel" if (args.finish_rows or args.prec == "bf16") else
                   ("fused matrix-core kernel" if args.prec == "fp16" else "none"),
                   **({"substitution_products": "FP32 matrix cores" if args.subst_fp32 else
                       "split FP16 (hi/lo) matrix cores"} if (sym and inv in (L.INV_CHOLESKY_APPLY_FP32, L.INV_CHOLESKY_FP32)) else {}),
                   **({"ns_tiles": tiles} if tiles else {}),
                   "parallelism": "single GPU"},
        "submatrices_per_s": round(system.nmol / (ms / 1e3), 1),
        "tflops_paper_count": round(tflops_paper, 3),
        "ns_iters": [int(it.min()), round(float(it.mean()), 2), int(it.max())],
        **({"inverse_iters": [int(iti.min()), round(float(iti.mean()), 2), int(iti.max())]}
           if args.inverse == "coupled_ns" else {}),
        "flop_count": ("value: the products as executed, n^2 (n + 1) per product of the symmetric "
                       "iteration (its unique half)" if sym else
                       "value: 2 n^3 per matrix product of the sign iteration, as executed")
                      + ", plus 12 n^2 per finishing product; tflops_paper_count: 2 n^3 per product "
                        "of the sign iteration (the paper's count, Sec. IV-B)",
        "status_ok": int((st["status"] == 0).sum()),
        "phases_ms": phases,
        "roofline": roofline,
        "composite_bound": composite,
    }
    if args.want_w:
        # T_J(W) columns: reads A_J (8 n^2 B) and Dcols_J, writes Wcols_J,
        # once per owned molecule
        wbytes = float((nown * (8.0 * n ** 2 + 96.0 * n)).sum())
        out["w_matrix"] = {"ms": round(prof["ms_wmat"], 3),
                           "GB_per_s": round(wbytes / (prof["ms_wmat"] / 1e3) / 1e9, 1) if prof["ms_wmat"] > 0 else None,
                           "bytes": wbytes}
    E_main = st["energy_KD"].copy()
    ex = sv.plan.export() if (args.density and lowp) else None
    Dm_host = sv.host_D() if ex is not None else None
    # the legs get the same workspace budget: the timed solver's goes first
    del sv
    torch.cuda.empty_cache()
    if args.legs and lowp:
        legs = {}
        if sym:
            leg, lms = time_leg(system, dev, args, "no_sym", args.leg_steps, prec=args.prec, sched=sched,
                                inverse=inv, sym_sign=0, ns_small_tile_mask=masks[False][0])
            lf = paper_and_exec_flops(leg, 0, system)
            legs["iteration_on_A"] = {
                "what": "the sign iteration on A_J = S_J^-1 K_J - mu I (no symmetric form), same batch",
                "steps": args.leg_steps, "ms_per_step": round(lms, 3),
                "tflops": round((lf["exec"] + lf["fin"]) / (lms / 1e3) / 1e12, 3),
                "submatrices_per_s": round(system.nmol / (lms / 1e3), 1),
                "ns_iters_mean": round(float(lf["it"].mean()), 2),
                "energy_max_diff_vs_main": float(np.abs(lf["st"]["energy_KD"] - E_main).max())}
            del leg
            torch.cuda.empty_cache()
        if sym and not args.combine:
            # the rescaling with learned spectral bounds (Sec. III-B.2): the
            # MLP is trained (untimed) with the library's kernels on the
            # stored, eigensolve-labelled features of a 4,096-molecule
            # trajectory of the same water-like model, then predicts the
            # bounds of every submatrix of this batch inside each step
            from paper_2104_08245_amd import learned
            ts = np.load(os.path.join(ROOT, "tests", "golden", "mlp_train_sym.npz"))
            tr = learned.train(ts["features"], ts["labels"], epochs=200, device=dev)
            torch.cuda.synchronize()
            leg, lms = time_leg(system, dev, args, "learned", args.leg_steps, prec=args.prec, sched=sched,
                                inverse=inv, sym_sign=1, ns_small_tile_mask=masks[True][0],
                                bounds=L.BOUNDS_LEARNED, d_mlp=tr["params"].data_ptr(),
                                d_mlp_norm=tr["norm"].data_ptr())
            lf = paper_and_exec_flops(leg, 1, system)
            legs["learned_bounds"] = {
                "what": "the main line with learned spectral bounds (MLP trained on stored eigensolve "
                        "labels of a 4,096-molecule trajectory of the same model), same batch",
                "steps": args.leg_steps, "ms_per_step": round(lms, 3),
                "submatrices_per_s": round(system.nmol / (lms / 1e3), 1),
                "ns_iters_mean": round(float(lf["it"].mean()), 2),
                "restarts": int(lf["st"]["fallback"].sum()),
                "status_ok": int((lf["st"]["status"] == 0).sum()),
                "energy_max_diff_vs_main": float(np.abs(lf["st"]["energy_KD"] - E_main).max())}
            E_learned = lf["st"]["energy_KD"].copy()
            del leg, tr
            torch.cuda.empty_cache()
        ref, fms = time_leg(system, dev, args, "fp64", args.fp64_steps, prec="fp64", sched=sched)
        rf = paper_and_exec_flops(ref, 0, system)
        ftf = (rf["exec"] + rf["fin"]) / (fms / 1e3) / 1e12
        legs["fp64_gpu"] = {
            "what": "plain FP64 GPU path (sign iteration on A_J to ||X^2 - I||_F < 1e-10), same batch",
            "steps": args.fp64_steps, "ms_per_step": round(fms, 3), "tflops": round(ftf, 3),
            "frac_of_fp64_peak": round(ftf / PEAK_TFLOPS["fp64"], 4),
            "submatrices_per_s": round(system.nmol / (fms / 1e3), 1),
            "ns_iters_mean": round(float(rf["it"].mean()), 2),
            "status_ok": int((rf["st"]["status"] == 0).sum())}
        e64 = rf["st"]["energy_KD"]
        dE = np.abs(E_main - e64)
        out["speedup_vs_fp64_gpu"] = round(fms / ms, 2)
        out["energy_error_vs_fp64_gpu"] = {"max": float(dE.max()), "mean": float(dE.mean()),
                                           "molecules": int(len(dE))}
        if "learned_bounds" in legs:
            legs["learned_bounds"]["energy_error_vs_fp64_gpu_max"] = float(np.abs(E_learned - e64).max())
        out["legs"] = legs
        if ex is not None:
            out["density_checks"] = density_against_fp64(system, ex, Dm_host, ref)
        del ref
        torch.cuda.empty_cache()
    if cpu is not None:
        dE = np.array([abs(E_main[J] - e) for J, e in cpu["E"].items()])
        out["energy_error_vs_oracle"] = {"max": float(dE.max()), "mean": float(dE.mean()),
                                         "molecules": int(len(dE))}
        one = cpu["single"]
        out["cpu_baseline"] = {"value": round(cpu["flops"] / cpu["wall"] / 1e12, 5), "unit": "TFLOP/s",
                               "cores": cpu["workers"], "kind": "oracle",
                               "sample": f"{cpu['n']} randomly chosen molecules of the same system, "
                                         f"FP64 oracle (2 n^3 per product as executed), one process per "
                                         f"core, {cpu['wall']:.1f}s wall",
                               "submatrices_per_s": round(cpu["n"] / cpu["wall"], 2),
                               "single_core": {"value": round(one["flops"] / one["wall"] / 1e12, 5),
                                               "submatrices_per_s": round(one["n"] / one["wall"], 3),
                                               "molecules": one["n"]},
                               "host_cpus": os.cpu_count(), "job_cpu_share": cpu["share"],
                               "cpu_model": cpu_model()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
