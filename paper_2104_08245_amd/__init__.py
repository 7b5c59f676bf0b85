"""MI355X-native NOLSM hot path (libnolsm.so + a ctypes binding).

The compute runs only in the HIP kernels of libnolsm.so; importing the
binding without the built library raises (there is no CPU fallback)."""
from . import _lib
from ._lib import NolsmError, default_opts, lib
from .nolsm import Plan, Solver, mlp_adam, mlp_forward, mlp_loss_grad

__all__ = ["Plan", "Solver", "NolsmError", "default_opts", "lib", "mlp_forward", "mlp_loss_grad",
           "mlp_adam", "_lib"]
