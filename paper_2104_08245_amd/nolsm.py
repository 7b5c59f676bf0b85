"""Python API over the C ABI. PyTorch only provides device memory and streams;
every step of the path runs in libnolsm.so's HIP kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


class Plan:
    """nolsm_build_submatrices (+ configure / bind). Host arrays are int32."""

    def __init__(self, nb, bs, K_row_ptr, K_col_idx, S_row_ptr=None, S_col_idx=None, flags=0):
        lib = L.lib()
        self._keep = [np.ascontiguousarray(K_row_ptr, np.int32), np.ascontiguousarray(K_col_idx, np.int32)]
        if S_row_ptr is None:
            S_row_ptr, S_col_idx = K_row_ptr, K_col_idx
        self._keep += [np.ascontiguousarray(S_row_ptr, np.int32), np.ascontiguousarray(S_col_idx, np.int32)]
        krp, kci, srp, sci = self._keep
        pk = L.Pattern(nb, bs, kci.shape[0], L.i32_ptr(krp), L.i32_ptr(kci))
        ps = L.Pattern(nb, bs, sci.shape[0], L.i32_ptr(srp), L.i32_ptr(sci))
        h = C.c_void_p()
        L.check(lib.nolsm_build_submatrices(C.byref(pk), C.byref(ps), flags, C.byref(h)))
        self.h = h
        self.nb, self.bs = nb, bs
        self.meta = None
        self.opts = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                L.lib().nolsm_plan_destroy(h)
            except Exception:
                pass
            self.h = None

    def info(self):
        s = L.PlanSizes()
        L.check(L.lib().nolsm_plan_info(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in L.PlanSizes._fields_}

    def export(self):
        inf = self.info()
        nb, sm = self.nb, inf["sum_m"]
        out = dict(sub_ptr=np.zeros(nb + 1, np.int32), sub_blk=np.zeros(sm, np.int32),
                   self_pos=np.zeros(nb, np.int32), D_row_ptr=np.zeros(nb + 1, np.int32),
                   D_col_idx=np.zeros(sm, np.int32), scatter_pos=np.zeros(sm, np.int32))
        L.check(L.lib().nolsm_plan_export(self.h, *[L.i32_ptr(out[k]) for k in
                                                    ("sub_ptr", "sub_blk", "self_pos", "D_row_ptr",
                                                     "D_col_idx", "scatter_pos")]))
        return out

    def groups(self):
        """(grp_ptr, grp_blk, own_ptr, own_J): the submatrices and the
        molecules each one owns (one per molecule unless combined)."""
        inf = self.info()
        ng = inf["ngroups"]
        out = (np.zeros(ng + 1, np.int32), np.zeros(inf["sum_gm"], np.int32),
               np.zeros(ng + 1, np.int32), np.zeros(self.nb, np.int32))
        L.check(L.lib().nolsm_plan_groups(self.h, *[L.i32_ptr(a) for a in out]))
        return out

    def configure(self, opts, ws_bytes):
        mb = C.c_size_t(0)
        L.check(L.lib().nolsm_plan_configure(self.h, C.byref(opts), int(ws_bytes), C.byref(mb)))
        self.opts = opts
        return mb.value

    def bind(self, meta_bytes, device, stream=None):
        torch = _torch()
        self.meta = torch.empty(max(int(meta_bytes), 256), dtype=torch.uint8, device=device)
        st = stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
        L.check(L.lib().nolsm_plan_bind(self.h, C.c_void_p(self.meta.data_ptr()), self.meta.numel(),
                                        C.c_void_p(st)))


def _stream_ptr(stream, device):
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream(device).cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Solver:
    """One system (K, S block-CSR) on one GPU: uploads the values, owns the
    workspace, metadata and outputs as torch tensors, runs nolsm_sign_batch."""

    def __init__(self, system, prec="fp64", device="cuda:0", ws_bytes=None, ws_budget=48 << 30,
                 combine=False, **opt_kw):
        torch = _torch()
        K, S = system.K, system.S
        self.device = torch.device(device)
        self.nb, self.bs = K.nb, K.bs
        self.plan = Plan(K.nb, K.bs, K.row_ptr, K.col_idx, S.row_ptr, S.col_idx,
                         flags=L.PLAN_COMBINE if combine else 0)
        self.opts = L.default_opts(prec, **opt_kw)
        full = self.plan.info()
        # first configure with the budget to learn the full size
        budget = int(ws_bytes) if ws_bytes is not None else int(ws_budget)
        mb = self.plan.configure(self.opts, budget)
        inf = self.plan.info()
        if ws_bytes is None:
            ws_bytes = min(budget, inf["ws_full_bytes"])
            mb = self.plan.configure(self.opts, ws_bytes)
        self.ws_bytes = int(ws_bytes)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.plan.bind(mb, self.device)
        self.sum_m = full["sum_m"]
        self.sum_n3 = full["sum_n3"]
        self.Kv = torch.from_numpy(np.ascontiguousarray(K.val).reshape(-1)).to(self.device)
        self.Sv = torch.from_numpy(np.ascontiguousarray(S.val).reshape(-1)).to(self.device)
        bsq = self.bs * self.bs
        self.Dcols = torch.zeros(self.sum_m * bsq, dtype=torch.float64, device=self.device)
        self.D = torch.zeros(self.sum_m * bsq, dtype=torch.float64, device=self.device)
        self.stats = torch.zeros(self.nb * C.sizeof(L.MolStats), dtype=torch.uint8, device=self.device)
        self.mu = system.mu
        self.features = None
        self.Wcols = None
        self.W = None

    def set_opts(self, **kw):
        for k, v in kw.items():
            setattr(self.opts, k, v)

    def reconfigure(self, **kw):
        """Options that change the plan's task lists or layout (the NS tile
        mask, the schedule): configure again within the same workspace and
        upload the new metadata."""
        self.set_opts(**kw)
        mb = self.plan.configure(self.opts, self.ws_bytes)
        self.plan.bind(mb, self.device)

    def want_w(self):
        """Also compute the owned columns of the energy-weighted density
        matrix T_J(W) = T_J(D) T_J(K) T_J(D) on every run (Sec. III-B.2)."""
        torch = _torch()
        n = self.sum_m * self.bs * self.bs
        self.Wcols = torch.zeros(n, dtype=torch.float64, device=self.device)
        self.W = torch.zeros(n, dtype=torch.float64, device=self.device)
        self.opts.d_wcols = self.Wcols.data_ptr()

    def want_features(self):
        torch = _torch()
        self.features = torch.zeros(self.nb * L.MLP_NFEAT, dtype=torch.float32, device=self.device)
        self.opts.d_features = self.features.data_ptr()

    def run(self, mu=None, stream=None, scatter=True):
        mu = self.mu if mu is None else mu
        st = _stream_ptr(stream, self.device)
        L.check(L.lib().nolsm_sign_batch(
            self.plan.h, C.c_void_p(self.Kv.data_ptr()), C.c_void_p(self.Sv.data_ptr()), float(mu),
            C.byref(self.opts), C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
            C.c_void_p(self.Dcols.data_ptr()), C.c_void_p(self.D.data_ptr() if scatter else None),
            C.c_void_p(self.stats.data_ptr()), C.c_void_p(st)))

    def run_noalloc(self, mu=None, stream=None, scatter=True):
        """nolsm_sign_batch_noalloc: the same solve with the library's static
        workspace array instead of self.ws (the plan must be configured for
        at most NOALLOC_WS_BYTES)."""
        mu = self.mu if mu is None else mu
        st = _stream_ptr(stream, self.device)
        L.check(L.lib().nolsm_sign_batch_noalloc(
            self.plan.h, C.c_void_p(self.Kv.data_ptr()), C.c_void_p(self.Sv.data_ptr()), float(mu),
            C.byref(self.opts), C.c_void_p(self.Dcols.data_ptr()),
            C.c_void_p(self.D.data_ptr() if scatter else None), C.c_void_p(self.stats.data_ptr()),
            C.c_void_p(st)))

    def trace_sums(self, stream=None):
        """(sum_J N_J, sum_J E_J, #molecules not OK) of the last solve, FP64 on the GPU."""
        out = (C.c_double * 3)()
        st = _stream_ptr(stream, self.device)
        L.check(L.lib().nolsm_trace_sums(self.plan.h, C.c_void_p(self.stats.data_ptr()),
                                         C.c_void_p(self.ws.data_ptr()), out, C.c_void_p(st)))
        return out[0], out[1], int(out[2])

    def mu_bisect(self, mu_lo, mu_hi, n_target, tol_count=0.5, max_steps=40, stream=None,
                  allow_noconv=False):
        """Chemical potential with sum_J N_J = n_target (bisection on the GPU
        solves). Returns (mu, count, steps). The library reports E_NOCONV when
        the count is not reached or some molecule of the final solve is not
        OK; that raises unless allow_noconv, which then returns
        (mu, count, steps, converged) with the last solve kept."""
        st = _stream_ptr(stream, self.device)
        mu, cnt, steps = C.c_double(), C.c_double(), C.c_int32()
        rc = L.lib().nolsm_mu_bisect(
            self.plan.h, C.c_void_p(self.Kv.data_ptr()), C.c_void_p(self.Sv.data_ptr()), float(mu_lo),
            float(mu_hi), float(n_target), float(tol_count), int(max_steps), C.byref(self.opts),
            C.c_void_p(self.ws.data_ptr()), self.ws_bytes, C.c_void_p(self.Dcols.data_ptr()),
            C.c_void_p(self.D.data_ptr()), C.c_void_p(self.stats.data_ptr()), C.c_void_p(st),
            C.byref(mu), C.byref(cnt), C.byref(steps))
        if allow_noconv:
            if rc not in (L.NOLSM_OK, L.E_NOCONV):
                L.check(rc)
            return mu.value, cnt.value, steps.value, rc == L.NOLSM_OK
        L.check(rc)
        return mu.value, cnt.value, steps.value

    def assemble(self, stream=None):
        st = _stream_ptr(stream, self.device)
        L.check(L.lib().nolsm_assemble_D(self.plan.h, C.c_void_p(self.Dcols.data_ptr()),
                                         C.c_void_p(self.D.data_ptr()), C.c_void_p(st)))

    def assemble_w(self, stream=None):
        """Write W back into D's block-CSR pattern (same scatter as D)."""
        st = _stream_ptr(stream, self.device)
        L.check(L.lib().nolsm_assemble_D(self.plan.h, C.c_void_p(self.Wcols.data_ptr()),
                                         C.c_void_p(self.W.data_ptr()), C.c_void_p(st)))

    def profile(self):
        """Phase times (ms) of the last run made with opts.profile = 1."""
        p = L.Profile()
        L.check(L.lib().nolsm_profile_last(self.plan.h, C.byref(p)))
        return {k: getattr(p, k) for k, _ in L.Profile._fields_}

    def host_stats(self):
        raw = self.stats.cpu().numpy()
        return raw.view(np.dtype(L.MOLSTATS_DTYPE))

    def host_dcols(self, which="D"):
        """List of (n_J, bs) arrays, one per molecule (which="W": T_J(W))."""
        flat = (self.Wcols if which == "W" else self.Dcols).cpu().numpy()
        ex = self.plan.export()
        sp = ex["sub_ptr"]
        bs = self.bs
        out = []
        for J in range(self.nb):
            a, b = sp[J] * bs * bs, sp[J + 1] * bs * bs
            out.append(flat[a:b].reshape(-1, bs))
        return out

    def host_D(self):
        return self.D.cpu().numpy().reshape(-1, self.bs, self.bs)


def mlp_forward(params, norm, x, out, stream=None):
    torch = _torch()
    st = _stream_ptr(stream, x.device)
    L.check(L.lib().nolsm_mlp_forward(C.c_void_p(params.data_ptr()), C.c_void_p(norm.data_ptr()),
                                      C.c_void_p(x.data_ptr()), int(x.shape[0]),
                                      C.c_void_p(out.data_ptr()), C.c_void_p(st)))


def mlp_loss_grad(params, norm, x, y, grad, loss, stream=None):
    st = _stream_ptr(stream, x.device)
    L.check(L.lib().nolsm_mlp_loss_grad(C.c_void_p(params.data_ptr()), C.c_void_p(norm.data_ptr()),
                                        C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), int(x.shape[0]),
                                        C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()),
                                        C.c_void_p(st)))


def mlp_adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    st = _stream_ptr(stream, params.device)
    L.check(L.lib().nolsm_mlp_adam(C.c_void_p(params.data_ptr()), C.c_void_p(grad.data_ptr()),
                                   C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()), int(t), float(lr),
                                   float(b1), float(b2), float(eps), C.c_void_p(st)))
