"""ctypes binding of the denoiser C ABI (include/sde_nn.h): argument
marshalling only.

Every layer, the loss, the gradients and the Adam update run in the HIP
kernels of ``libsde.so``; torch provides the device tensors.  bf16 operands
are passed as ``torch.bfloat16`` tensors (their bit patterns are what the
kernels read).
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import numpy as np

from . import sde
from .sde import _check, lib

EXPORTS = ("sde_nn_create", "sde_nn_destroy", "sde_nn_param_count", "sde_nn_set_params",
           "sde_nn_get_params", "sde_nn_set_adam_state", "sde_nn_get_adam_state",
           "sde_nn_get_grads", "sde_nn_forward", "sde_nn_loss_grad", "sde_nn_adam_step",
           "sde_nn_denoise", "sde_nn_prepare_pair", "sde_nn_conv3d_fwd", "sde_nn_conv3d_workspace",
           "sde_nn_conv3d_dgrad", "sde_nn_conv3d_wgrad")


class Config(C.Structure):
    _fields_ = [("levels", C.c_int), ("base_channels", C.c_int), ("in_channels", C.c_int),
                ("leaky_alpha", C.c_float), ("max_batch", C.c_int), ("max_d", C.c_int),
                ("max_h", C.c_int), ("max_w", C.c_int), ("train", C.c_int),
                ("adam_beta1", C.c_float), ("adam_beta2", C.c_float), ("adam_eps", C.c_float),
                ("store_concat", C.c_int)]


def _setup():
    P, V, I, F = C.POINTER, C.c_void_p, C.c_int, C.c_float
    i64 = C.c_int64
    lib.sde_nn_create.argtypes = [P(Config), P(V)]
    lib.sde_nn_destroy.argtypes = [V]
    lib.sde_nn_param_count.argtypes = [V, P(i64)]
    lib.sde_nn_set_params.argtypes = [V, V, i64]
    lib.sde_nn_get_params.argtypes = [V, V, i64]
    lib.sde_nn_set_adam_state.argtypes = [V, V, V, i64, i64]
    lib.sde_nn_get_adam_state.argtypes = [V, V, V, i64, P(i64)]
    lib.sde_nn_get_grads.argtypes = [V, V, i64]
    lib.sde_nn_forward.argtypes = [V, V, V, I, I, I, I, V]
    lib.sde_nn_loss_grad.argtypes = [V, V, V, V, V, I, I, I, I, P(F)]
    lib.sde_nn_adam_step.argtypes = [V, F]
    lib.sde_nn_denoise.argtypes = [V, V, V, I, I, I, V]
    lib.sde_nn_prepare_pair.argtypes = [V, V, V, i64, F, F, V, V, V]
    lib.sde_nn_conv3d_fwd.argtypes = [V, V, V, I, I, I, I, I, I, F, I, V, V]
    lib.sde_nn_conv3d_workspace.argtypes = [I, I, I, I, I, I, P(C.c_size_t)]
    lib.sde_nn_conv3d_dgrad.argtypes = [V, V, I, I, I, I, I, I, V, V, C.c_size_t]
    lib.sde_nn_conv3d_wgrad.argtypes = [V, V, I, I, I, I, I, I, V, V, V, C.c_size_t]
    for name in EXPORTS:
        getattr(lib, name).restype = C.c_int


_setup()


def _p(t) -> Optional[int]:
    return None if t is None else sde._dptr(t)


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


class Net:
    """A denoiser network with its device buffers (see include/sde_nn.h)."""

    def __init__(self, levels: int = 4, base_channels: int = 16, in_channels: int = 16,
                 alpha: float = 0.01, max_batch: int = 1, max_dims: Tuple[int, int, int] = (64, 64, 64),
                 train: bool = False, betas=(0.9, 0.999), eps: float = 1e-8,
                 store_concat: bool = False):
        cfg = Config(levels, base_channels, in_channels, alpha, max_batch, *max_dims, int(train),
                     betas[0], betas[1], eps, int(store_concat))
        h = C.c_void_p()
        _check(lib.sde_nn_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self.levels, self.c0, self.cin, self.alpha = levels, base_channels, in_channels, alpha
        n = C.c_int64()
        _check(lib.sde_nn_param_count(h, C.byref(n)))
        self.n_params = int(n.value)

    def close(self):
        if self._h:
            _check(lib.sde_nn_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # parameters and optimiser state -------------------------------------
    def set_params(self, p: np.ndarray):
        p = _f32(p)
        _check(lib.sde_nn_set_params(self._h, p.ctypes.data, p.size))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, np.float32)
        _check(lib.sde_nn_get_params(self._h, p.ctypes.data, p.size))
        return p

    def get_grads(self) -> np.ndarray:
        g = np.empty(self.n_params, np.float32)
        _check(lib.sde_nn_get_grads(self._h, g.ctypes.data, g.size))
        return g

    def set_adam_state(self, m: np.ndarray, v: np.ndarray, step: int):
        m, v = _f32(m), _f32(v)
        _check(lib.sde_nn_set_adam_state(self._h, m.ctypes.data, v.ctypes.data, m.size, step))

    def get_adam_state(self):
        m = np.empty(self.n_params, np.float32)
        v = np.empty(self.n_params, np.float32)
        s = C.c_int64()
        _check(lib.sde_nn_get_adam_state(self._h, m.ctypes.data, v.ctypes.data, m.size,
                                         C.byref(s)))
        return m, v, int(s.value)

    # compute -------------------------------------------------------------
    def forward(self, dose, rho, out):
        """dose, rho (nullable), out: float32 device tensors (B, D, H, W)."""
        B, D, H, W = dose.shape
        _check(lib.sde_nn_forward(self._h, _p(dose), _p(rho), B, D, H, W, _p(out)))

    def loss_grad(self, dose, rho, target, weight=None) -> float:
        B, D, H, W = dose.shape
        loss = C.c_float()
        _check(lib.sde_nn_loss_grad(self._h, _p(dose), _p(rho), _p(target), _p(weight), B, D, H,
                                    W, C.byref(loss)))
        return float(loss.value)

    def adam_step(self, lr: float):
        _check(lib.sde_nn_adam_step(self._h, lr))

    def denoise(self, dose, rho, out):
        """dose, out: float64 device tensors (nz, ny, nx); rho float32 or None."""
        nz, ny, nx = dose.shape
        _check(lib.sde_nn_denoise(self._h, _p(dose), _p(rho), nx, ny, nz, _p(out)))

    def prepare_pair(self, low, high, low_out, high_out=None, weight_out=None,
                     eps: float = 0.02, thr: float = 0.01):
        """Normalise a (low, high) pair of FP64 device dose grids by max |low|."""
        _check(lib.sde_nn_prepare_pair(self._h, _p(low), _p(high), low.numel(), eps, thr,
                                       _p(low_out), _p(high_out), _p(weight_out)))


# single layers (kernel tests) --------------------------------------------

def conv3d_fwd(x, w, bias, alpha: float = 0.01, act: bool = True, out16=None, out32=None):
    """x: bf16 (B, D, H, W, Ci); w: bf16 (Co, 27, Ci); bias float32 (Co,) or None."""
    B, D, H, W, Ci = x.shape
    Co = w.shape[0]
    _check(lib.sde_nn_conv3d_fwd(_p(x), _p(w), _p(bias), B, D, H, W, Ci, Co, alpha, int(act),
                                 _p(out16), _p(out32)))


def _workspace(B, D, H, W, Ci, Co):
    import torch
    n = C.c_size_t()
    _check(lib.sde_nn_conv3d_workspace(B, D, H, W, Ci, Co, C.byref(n)))
    return torch.empty(max(int(n.value), 1), dtype=torch.uint8, device="cuda"), int(n.value)


def conv3d_dgrad(dz, w, dx):
    """dz: bf16 (B, D, H, W, Co); w: bf16 (Co, 27, Ci); dx: float32 (B, D, H, W, Ci)."""
    B, D, H, W, Co = dz.shape
    Ci = w.shape[2]
    ws, nb = _workspace(B, D, H, W, Ci, Co)
    _check(lib.sde_nn_conv3d_dgrad(_p(dz), _p(w), B, D, H, W, Ci, Co, _p(dx), _p(ws), nb))


def conv3d_wgrad(dz, x, dw, db=None):
    """dz: bf16 (B, D, H, W, Co); x: bf16 (B, D, H, W, Ci); dw float32 (Co, 27, Ci)."""
    B, D, H, W, Co = dz.shape
    Ci = x.shape[4]
    ws, nb = _workspace(B, D, H, W, Ci, Co)
    _check(lib.sde_nn_conv3d_wgrad(_p(dz), _p(x), B, D, H, W, Ci, Co, _p(dw), _p(db), _p(ws), nb))
