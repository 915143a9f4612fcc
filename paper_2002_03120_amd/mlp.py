"""Python binding of the surrogate MLP's C ABI (include/sdpdem_mlp.h),
argument marshalling only: every computation runs in the HIP kernels of
libsdpdem.so."""
from __future__ import annotations

import ctypes

import numpy as np

from . import sdpdem as S

NPARAMS = 8705
MAX_BATCH = 256


class MlpConfig(ctypes.Structure):
    _fields_ = [
        ("norm_mean", ctypes.c_float * 4), ("norm_std", ctypes.c_float * 4),
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float), ("max_batch", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_bound = False


def lib():
    global _bound
    L = S.lib()
    if not _bound:
        vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
        L.sdpdem_mlp_workspace_bytes.argtypes = [ctypes.POINTER(MlpConfig), ctypes.POINTER(sz)]
        L.sdpdem_mlp_create.argtypes = [ctypes.POINTER(MlpConfig), vp, vp, sz, vp,
                                        ctypes.POINTER(vp)]
        L.sdpdem_mlp_predict.argtypes = [vp, vp, vp, i64, vp]
        L.sdpdem_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp]
        L.sdpdem_mlp_read.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
        L.sdpdem_mlp_destroy.argtypes = [vp]
        L.sdpdem_mlp_destroy.restype = None
        _bound = True
    return L


def make_config(norm, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, max_batch=MAX_BATCH):
    c = MlpConfig()
    for f in range(4):
        c.norm_mean[f] = float(norm[f])
        c.norm_std[f] = float(norm[4 + f])
    c.lr, c.beta1, c.beta2, c.eps = lr, beta1, beta2, eps
    c.max_batch = int(max_batch)
    c.reserved = 0
    return c


def sdpdem_mlp_workspace_bytes(cfg: MlpConfig) -> int:
    out = ctypes.c_size_t()
    S._check(lib().sdpdem_mlp_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)),
             "sdpdem_mlp_workspace_bytes")
    return int(out.value)


class Mlp:
    """The surrogate network in a device workspace (torch uint8 tensor)."""

    def __init__(self, init_params, norm, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 max_batch=MAX_BATCH, stream=None):
        import torch
        self.cfg = make_config(norm, lr, beta1, beta2, eps, max_batch)
        self.stream = stream
        self.workspace = torch.empty(sdpdem_mlp_workspace_bytes(self.cfg), dtype=torch.uint8,
                                     device="cuda")
        p = np.ascontiguousarray(init_params, dtype=np.float32)
        if p.size != NPARAMS:
            raise ValueError(f"expected {NPARAMS} parameters")
        h = ctypes.c_void_p()
        S._check(lib().sdpdem_mlp_create(ctypes.byref(self.cfg), p.ctypes.data,
                                         ctypes.c_void_p(self.workspace.data_ptr()),
                                         self.workspace.numel(), S._stream(stream),
                                         ctypes.byref(h)), "sdpdem_mlp_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().sdpdem_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def predict(self, x, y=None):
        """x: device float32 tensor [n, 4]; returns a device tensor [n]."""
        import torch
        x = x.contiguous()
        if y is None:
            y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        S._check(lib().sdpdem_mlp_predict(self.h, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(y.data_ptr()), x.shape[0],
                                          S._stream(self.stream)), "sdpdem_mlp_predict")
        return y

    def train_step(self, x, t, update=True):
        x = x.contiguous()
        t = t.contiguous()
        S._check(lib().sdpdem_mlp_train_step(self.h, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(t.data_ptr()), x.shape[0],
                                             1 if update else 0, S._stream(self.stream)),
                 "sdpdem_mlp_train_step")

    def read(self):
        """(master params, params as used, last gradient, last loss, Adam steps)"""
        p = np.empty(NPARAMS, np.float32)
        q = np.empty(NPARAMS, np.float32)
        g = np.empty(NPARAMS, np.float32)
        loss = np.empty(1, np.float32)
        steps = ctypes.c_int64()
        S._check(lib().sdpdem_mlp_read(self.h, p.ctypes.data, q.ctypes.data, g.ctypes.data,
                                       loss.ctypes.data, ctypes.byref(steps),
                                       S._stream(self.stream)), "sdpdem_mlp_read")
        return p, q, g, float(loss[0]), int(steps.value)
