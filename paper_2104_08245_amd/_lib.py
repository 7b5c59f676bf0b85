"""ctypes binding of libnolsm.so: the same entry points as include/nolsm.h,
argument marshalling only. Raises if the library has not been built."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# NOLSM_LIB names another build of the library (the AddressSanitizer build
# of the host plan code used by a CPU test): only the symbols it has are bound
LIB_OVERRIDE = os.environ.get("NOLSM_LIB")
LIB_PATH = LIB_OVERRIDE or os.path.join(HERE, "libnolsm.so")

NOLSM_OK = 0
E_ARG, E_PATTERN, E_WORKSPACE, E_HIP, E_STATE, E_NOT_SPD, E_NOCONV, E_NOMEM = range(-1, -9, -1)
MOL_OK, MOL_NOT_SPD, MOL_NOCONV = 0, 1, 2
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}
BOUNDS_GERSHGORIN, BOUNDS_LEARNED = 0, 1
SCHED_GRAPH, SCHED_STREAM, SCHED_PER_BUCKET, SCHED_PERSISTENT, SCHED_PIPELINE = 0, 1, 2, 3, 4
INV_CHOLESKY, INV_COUPLED_NS, INV_CHOLESKY_FP32, INV_CHOLESKY_APPLY_FP32 = 0, 1, 2, 3
PLAN_COMBINE = 1
NOALLOC_WS_BYTES = 64 << 20   # NOLSM_NOALLOC_WS_BYTES
MAX_ROWS = 3008               # NOLSM_MAX_ROWS
MLP_NFEAT = 12
MLP_NPARAM = 5122


class NolsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nolsm error {code}: {msg}")
        self.code = code


class Pattern(C.Structure):
    _fields_ = [("nb", C.c_int32), ("bs", C.c_int32), ("nnzb", C.c_int64),
                ("row_ptr", C.POINTER(C.c_int32)), ("col_idx", C.POINTER(C.c_int32))]


class SolveOpts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("n_final_fp32", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("fixed_iters", C.c_int32),
                ("switch_theta", C.c_double), ("switch_rmax", C.c_double),
                ("bounds", C.c_int32), ("d_mlp", C.c_void_p), ("d_mlp_norm", C.c_void_p),
                ("mlp_safety", C.c_float), ("sched", C.c_int32), ("sync_errors", C.c_int32),
                ("d_features", C.c_void_p), ("debug_scale_mult", C.c_double),
                ("debug_poison_mol", C.c_int32), ("profile", C.c_int32),
                ("ns_small_tile_mask", C.c_uint64), ("d_wcols", C.c_void_p),
                ("inverse", C.c_int32), ("inv_max_iter", C.c_int32),
                ("sym_sign", C.c_int32), ("finish_rows", C.c_int32),
                ("debug_force_stall", C.c_int32), ("subst_fp32", C.c_int32)]


class MolStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("iters_fp32", C.c_int32), ("fallback", C.c_int32),
                ("status", C.c_int32), ("scale", C.c_double), ("resid", C.c_double),
                ("trace_SD", C.c_double), ("energy_KD", C.c_double),
                ("iters_inv", C.c_int32), ("reserved_", C.c_int32)]


MOLSTATS_DTYPE = [("iters", "<i4"), ("iters_fp32", "<i4"), ("fallback", "<i4"), ("status", "<i4"),
                  ("scale", "<f8"), ("resid", "<f8"), ("trace_SD", "<f8"), ("energy_KD", "<f8"),
                  ("iters_inv", "<i4"), ("reserved_", "<i4")]


class PlanSizes(C.Structure):
    _fields_ = [("nb", C.c_int32), ("bs", C.c_int32), ("sum_m", C.c_int64),
                ("m_min", C.c_int32), ("m_max", C.c_int32), ("sum_n3", C.c_double),
                ("nchunks", C.c_int32), ("meta_bytes", C.c_size_t),
                ("ws_min_bytes", C.c_size_t), ("ws_full_bytes", C.c_size_t),
                ("ngroups", C.c_int32), ("g_m_max", C.c_int32), ("sum_gm", C.c_int64),
                ("sum_gn3", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("valid", C.c_int32), ("nchunks", C.c_int32), ("n_ns_launches", C.c_int32),
                ("n_fin_launches", C.c_int32), ("ms_gather", C.c_double), ("ms_chol", C.c_double),
                ("ms_subst", C.c_double), ("ms_bounds", C.c_double), ("ms_ns", C.c_double),
                ("ms_finish", C.c_double), ("ms_extract", C.c_double), ("ms_total", C.c_double),
                ("ms_wmat", C.c_double), ("ms_inverse", C.c_double)]


EXPORTED = ["nolsm_default_opts", "nolsm_build_submatrices", "nolsm_plan_info", "nolsm_plan_export",
            "nolsm_plan_configure", "nolsm_plan_bind", "nolsm_sign_batch", "nolsm_assemble_D",
            "nolsm_plan_destroy", "nolsm_strerror", "nolsm_mlp_forward", "nolsm_mlp_loss_grad",
            "nolsm_mlp_adam", "nolsm_profile_last", "nolsm_trace_sums", "nolsm_mu_bisect",
            "nolsm_plan_groups", "nolsm_switch_tol", "nolsm_sign_batch_noalloc"]

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2104_08245_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    p_i32 = C.POINTER(C.c_int32)
    sigs = {
        "nolsm_default_opts": ([C.POINTER(SolveOpts), i32], None),
        "nolsm_switch_tol": ([i32, i32, dbl], dbl),
        "nolsm_build_submatrices": ([C.POINTER(Pattern), C.POINTER(Pattern), i32, C.POINTER(vp)], C.c_int),
        "nolsm_plan_info": ([vp, C.POINTER(PlanSizes)], C.c_int),
        "nolsm_plan_export": ([vp, p_i32, p_i32, p_i32, p_i32, p_i32, p_i32], C.c_int),
        "nolsm_plan_groups": ([vp, p_i32, p_i32, p_i32, p_i32], C.c_int),
        "nolsm_plan_configure": ([vp, C.POINTER(SolveOpts), sz, C.POINTER(sz)], C.c_int),
        "nolsm_plan_bind": ([vp, vp, sz, vp], C.c_int),
        "nolsm_sign_batch": ([vp, vp, vp, dbl, C.POINTER(SolveOpts), vp, sz, vp, vp, vp, vp], C.c_int),
        "nolsm_sign_batch_noalloc": ([vp, vp, vp, dbl, C.POINTER(SolveOpts), vp, vp, vp, vp], C.c_int),
        "nolsm_assemble_D": ([vp, vp, vp, vp], C.c_int),
        "nolsm_plan_destroy": ([vp], None),
        "nolsm_strerror": ([C.c_int], C.c_char_p),
        "nolsm_profile_last": ([vp, C.POINTER(Profile)], C.c_int),
        "nolsm_trace_sums": ([vp, vp, vp, C.POINTER(C.c_double), vp], C.c_int),
        "nolsm_mu_bisect": ([vp, vp, vp, dbl, dbl, dbl, dbl, i32, C.POINTER(SolveOpts), vp, sz, vp, vp,
                             vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)],
                            C.c_int),
        "nolsm_mlp_forward": ([vp, vp, vp, i32, vp, vp], C.c_int),
        "nolsm_mlp_loss_grad": ([vp, vp, vp, vp, i32, vp, vp, vp], C.c_int),
        "nolsm_mlp_adam": ([vp, vp, vp, vp, i32, C.c_double, C.c_double, C.c_double, C.c_double, vp], C.c_int),
    }
    assert set(sigs) == set(EXPORTED)
    for name in EXPORTED:
        if LIB_OVERRIDE and not hasattr(L, name):
            continue
        f = getattr(L, name)   # the library itself must export every symbol
        f.argtypes, f.restype = sigs[name]
    _lib = L
    return L


def check(rc):
    if rc != NOLSM_OK:
        raise NolsmError(rc, lib().nolsm_strerror(rc).decode())
    return rc


def i32_ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def default_opts(prec="fp64", **kw):
    o = SolveOpts()
    lib().nolsm_default_opts(C.byref(o), PREC[prec] if isinstance(prec, str) else int(prec))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o
