"""Training of the spectral-bound MLP on the GPU with the library's own
forward / loss-gradient / Adam kernels (nolsm_mlp_*). The host only shuffles
indices and moves batches; every forward and backward pass runs in
libnolsm.so.

Targets are the normalised extremes (lambda_min / G_lo, lambda_max / G_hi),
with [G_lo, G_hi] the intersection of the row and column Gershgorin
intervals taken from the features (features 7-10)."""
from __future__ import annotations

import numpy as np

from . import _lib as L
from .nolsm import mlp_adam, mlp_forward, mlp_loss_grad

NPARAM = L.MLP_NPARAM


def gershgorin_box(F):
    F = np.asarray(F, np.float64)
    return np.maximum(F[:, 7], F[:, 9]), np.minimum(F[:, 8], F[:, 10])


def targets(F, labels):
    glo, ghi = gershgorin_box(F)
    return np.stack([labels[:, 0] / glo, labels[:, 1] / ghi], axis=1)


def init_params(rng):
    """He-style uniform initialisation, zero biases (packing of nolsm.h)."""
    th = np.zeros(NPARAM)
    o = 0
    for shape in [(64, 12), (64,), (64, 64), (64,), (2, 64), (2,)]:
        k = int(np.prod(shape))
        if len(shape) == 2:
            th[o:o + k] = rng.uniform(-1, 1, k) * np.sqrt(3.0 / shape[1])
        o += k
    return th


def train(F, labels, epochs=200, batch=256, lr=1e-3, seed=0, val_frac=0.1, device="cuda:0", log=None):
    """Returns dict(params, norm, history) with params/norm as float32 torch
    tensors on `device` (ready for opts.d_mlp / opts.d_mlp_norm)."""
    import torch
    rng = np.random.default_rng(seed)
    F = np.asarray(F, np.float64)
    Y = targets(F, np.asarray(labels, np.float64))
    ok = np.all(np.isfinite(Y), axis=1) & (Y[:, 0] > 0) & (Y[:, 1] > 0)
    F, Y = F[ok], Y[ok]
    perm = rng.permutation(len(F))
    nval = int(len(F) * val_frac)
    va, tr = perm[:nval], perm[nval:]
    mean = F[tr].mean(0)
    std = F[tr].std(0) + 1e-6
    dev = torch.device(device)
    T = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)
    Xtr, Ytr, Xva, Yva = T(F[tr]), T(Y[tr]), T(F[va]), T(Y[va])
    norm = T(np.concatenate([mean, std]))
    params = T(init_params(rng))
    m = torch.zeros(NPARAM, device=dev)
    v = torch.zeros(NPARAM, device=dev)
    grad = torch.zeros(NPARAM, device=dev)
    loss = torch.zeros(1, device=dev)
    hist = []
    step = 0
    ntr = len(tr)
    for ep in range(epochs):
        order = torch.tensor(rng.permutation(ntr), device=dev)
        for s in range(0, ntr - batch + 1, batch):
            idx = order[s:s + batch]
            xb = Xtr.index_select(0, idx).contiguous()
            yb = Ytr.index_select(0, idx).contiguous()
            mlp_loss_grad(params, norm, xb, yb, grad, loss)
            step += 1
            mlp_adam(params, grad, m, v, step, lr=lr)
        if ep % 20 == 0 or ep == epochs - 1:
            mlp_loss_grad(params, norm, Xva, Yva, grad, loss) if len(va) else None
            vl = float(loss.item()) if len(va) else float("nan")
            hist.append((ep, vl))
            if log:
                log(f"epoch {ep}: validation loss {vl:.5f}")
    return dict(params=params, norm=norm, history=hist, mean=mean, std=std)


def predict(params, norm, F, device="cuda:0"):
    import torch
    x = torch.tensor(np.ascontiguousarray(F, np.float32), device=device)
    out = torch.zeros(len(F), 2, device=device)
    mlp_forward(params, norm, x, out)
    return out.cpu().numpy()
