"""Thin Python binding of the warm-start network's C ABI (``include/bte_mlp.h``).

Argument marshalling only: the forward pass, the loss gradient, the Adam
step and the normalisation statistics all run in ``libbte.so``.  PyTorch
provides device memory and the stream.  The training loop here only draws
the per-epoch row order (seeded) and hands index arrays to the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import bte as _bte

HEADER_PATH = os.path.join(os.path.dirname(_bte.HEADER_PATH), "bte_mlp.h")
BTE_MLP_IN, BTE_MLP_HIDDEN, BTE_MLP_OUT = 5, 256, 8192
BTE_MLP_BF16, BTE_MLP_FP32 = 0, 1

_lib = _bte.lib()
_vp, _fp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int32
for _name, (_args, _res) in {
    "bte_mlp_param_count": ([], ctypes.c_int64),
    "bte_mlp_workspace_bytes": ([_ip, _ip], ctypes.c_size_t),
    "bte_mlp_create": ([_ip, _ip, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "bte_mlp_set_params": ([_vp, _vp], ctypes.c_int),
    "bte_mlp_get_params": ([_vp, _vp], ctypes.c_int),
    "bte_mlp_fit_normalization": ([_vp, _vp, _vp, _ip], ctypes.c_int),
    "bte_mlp_get_normalization": ([_vp, _fp], ctypes.c_int),
    "bte_mlp_set_normalization": ([_vp, _fp], ctypes.c_int),
    "bte_mlp_forward": ([_vp, _vp, _ip, _vp], ctypes.c_int),
    "bte_mlp_loss_grad": ([_vp, _vp, _vp, _ip, _vp, _ip, _vp, _vp], ctypes.c_int),
    "bte_mlp_train_step": ([_vp, _vp, _vp, _ip, _vp, _ip, ctypes.c_float, _vp], ctypes.c_int),
    "bte_mlp_destroy": ([_vp], None),
}.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def _check(rc, func):
    _bte._check(rc, func)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---- the C entry points, same names --------------------------------------
def bte_mlp_param_count() -> int:
    return int(_lib.bte_mlp_param_count())


def bte_mlp_workspace_bytes(max_batch: int, precision: int) -> int:
    return int(_lib.bte_mlp_workspace_bytes(int(max_batch), int(precision)))


def bte_mlp_create(max_batch, precision, workspace_ptr, workspace_bytes, stream_ptr) -> int:
    h = ctypes.c_void_p()
    _check(_lib.bte_mlp_create(int(max_batch), int(precision), ctypes.c_void_p(workspace_ptr),
                               workspace_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(h)),
           "bte_mlp_create")
    return h.value


def bte_mlp_set_params(h, params):
    _check(_lib.bte_mlp_set_params(ctypes.c_void_p(h), _p(params)), "bte_mlp_set_params")


def bte_mlp_get_params(h, out):
    _check(_lib.bte_mlp_get_params(ctypes.c_void_p(h), _p(out)), "bte_mlp_get_params")


def bte_mlp_fit_normalization(h, features, coeffs, n):
    _check(_lib.bte_mlp_fit_normalization(ctypes.c_void_p(h), _p(features), _p(coeffs), int(n)),
           "bte_mlp_fit_normalization")


def bte_mlp_get_normalization(h) -> np.ndarray:
    out = (ctypes.c_float * 11)()
    _check(_lib.bte_mlp_get_normalization(ctypes.c_void_p(h), out), "bte_mlp_get_normalization")
    return np.array(out[:], dtype=np.float32)


def bte_mlp_set_normalization(h, values):
    v = (ctypes.c_float * 11)(*[float(x) for x in values])
    _check(_lib.bte_mlp_set_normalization(ctypes.c_void_p(h), v), "bte_mlp_set_normalization")


def bte_mlp_forward(h, features, n, out):
    _check(_lib.bte_mlp_forward(ctypes.c_void_p(h), _p(features), int(n), _p(out)),
           "bte_mlp_forward")


def bte_mlp_loss_grad(h, features, coeffs, n_rows, index, n, grad, loss):
    _check(_lib.bte_mlp_loss_grad(ctypes.c_void_p(h), _p(features), _p(coeffs), int(n_rows),
                                  _p(index), int(n), _p(grad), _p(loss)), "bte_mlp_loss_grad")


def bte_mlp_train_step(h, features, coeffs, n_rows, index, n, lr, loss):
    _check(_lib.bte_mlp_train_step(ctypes.c_void_p(h), _p(features), _p(coeffs), int(n_rows),
                                   _p(index), int(n), float(lr), _p(loss)), "bte_mlp_train_step")


def bte_mlp_destroy(h):
    _lib.bte_mlp_destroy(ctypes.c_void_p(h))


# ---- convenience wrapper ---------------------------------------------------
def features_of(instances):
    """n x 5 float32 array (E_dc, E_w, omega, B, mu) of workload-like objects."""
    return np.array([[w.E_dc, w.E_w, w.omega, w.B, w.mu] for w in instances], dtype=np.float32)


class Mlp:
    """The warm-start network on one device (see include/bte_mlp.h)."""

    def __init__(self, max_batch=512, precision=BTE_MLP_BF16, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.device = device
        self.max_batch = int(max_batch)
        self.precision = int(precision)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        nbytes = bte_mlp_workspace_bytes(self.max_batch, self.precision)
        if nbytes == 0:
            raise ValueError("invalid max_batch or precision")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.handle = bte_mlp_create(self.max_batch, self.precision, ptr, nbytes,
                                     self.stream.cuda_stream)
        self.n_params = bte_mlp_param_count()
        self._loss = torch.zeros(1, dtype=torch.float32, device=device)

    def _dev(self, a, dtype=None):
        t = self.torch.as_tensor(a, device=self.device)
        if dtype is not None:
            t = t.to(dtype)
        return t.contiguous()

    def set_params(self, params):
        p = self._dev(params, self.torch.float32).reshape(-1)
        assert p.numel() == self.n_params
        bte_mlp_set_params(self.handle, p)
        self.stream.synchronize()

    def params(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        bte_mlp_get_params(self.handle, out)
        self.stream.synchronize()
        return out

    def fit_normalization(self, features, coeffs):
        x = self._dev(features, self.torch.float32).reshape(-1, BTE_MLP_IN)
        c = self._dev(coeffs, self.torch.float32).reshape(x.shape[0], BTE_MLP_OUT)
        bte_mlp_fit_normalization(self.handle, x, c, x.shape[0])
        self.stream.synchronize()

    def normalization(self):
        return bte_mlp_get_normalization(self.handle)

    def set_normalization(self, values):
        bte_mlp_set_normalization(self.handle, values)

    def predict(self, features, out=None):
        """(n, 64, 128) float32 CUDA tensor of predicted coefficients."""
        x = self._dev(features, self.torch.float32).reshape(-1, BTE_MLP_IN)
        n = x.shape[0]
        if out is None:
            out = self.torch.empty((n, 64, 128), dtype=self.torch.float32, device=self.device)
        bte_mlp_forward(self.handle, x, n, out)
        self.stream.synchronize()
        return out

    def loss_grad(self, features, coeffs, index=None):
        x = self._dev(features, self.torch.float32).reshape(-1, BTE_MLP_IN)
        c = self._dev(coeffs, self.torch.float32).reshape(x.shape[0], BTE_MLP_OUT)
        idx = None if index is None else self._dev(index, self.torch.int32)
        n = x.shape[0] if idx is None else idx.numel()
        grad = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        bte_mlp_loss_grad(self.handle, x, c, x.shape[0], idx, n, grad, self._loss)
        self.stream.synchronize()
        return float(self._loss.item()), grad

    def train_step(self, features, coeffs, lr, index=None):
        x = self._dev(features, self.torch.float32).reshape(-1, BTE_MLP_IN)
        c = self._dev(coeffs, self.torch.float32).reshape(x.shape[0], BTE_MLP_OUT)
        idx = None if index is None else self._dev(index, self.torch.int32)
        n = x.shape[0] if idx is None else idx.numel()
        bte_mlp_train_step(self.handle, x, c, x.shape[0], idx, n, lr, self._loss)
        self.stream.synchronize()
        return float(self._loss.item())

    def train(self, features, coeffs, epochs, batch=256, lr=1e-3, lr_final=1e-5, seed=0,
              log=None, log_every=10):
        """Adam over `epochs` passes of shuffled mini-batches (the last partial
        batch of an epoch is dropped), with the learning rate decaying
        geometrically from lr to lr_final.  Returns the mean loss per epoch."""
        torch = self.torch
        x = self._dev(features, torch.float32).reshape(-1, BTE_MLP_IN)
        c = self._dev(coeffs, torch.float32).reshape(x.shape[0], BTE_MLP_OUT)
        n = x.shape[0]
        batch = min(batch, self.max_batch, n)
        per_epoch = n // batch
        total = max(1, epochs * per_epoch)
        g = np.random.Generator(np.random.PCG64(seed))
        losses = torch.zeros(total, dtype=torch.float32, device=self.device)
        step = 0
        history = []
        for e in range(epochs):
            order = torch.as_tensor(g.permutation(n).astype(np.int32), device=self.device)
            for b in range(per_epoch):
                rate = lr * (lr_final / lr) ** (step / max(1, total - 1))
                bte_mlp_train_step(self.handle, x, c, n, order[b * batch:(b + 1) * batch], batch,
                                   rate, losses[step:step + 1])
                step += 1
            self.stream.synchronize()
            history.append(float(losses[step - per_epoch:step].mean().item()))
            if log and (e % log_every == 0 or e == epochs - 1):
                log(f"  epoch {e}: loss {history[-1]:.4e}", flush=True)
        return history

    def close(self):
        if getattr(self, "handle", None):
            bte_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
