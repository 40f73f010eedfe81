"""ctypes binding of the surrogate network (include/hsc_mlp.h).

Argument marshalling only: forward, backward and Adam run in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .hsc import Context, check, lib, _dptr


class TrainOpts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("batch", C.c_int32), ("steps", C.c_int32)]


class MLP:
    """FP32 network widths[0] -> ... -> widths[-1], tanh hidden layers, on the context's device."""

    def __init__(self, ctx: Context, widths):
        self.ctx = ctx
        self.widths = [int(w) for w in widths]
        w = np.asarray(self.widths, np.int32)
        h = C.c_void_p()
        check(lib().hsc_mlp_create(ctx.h, len(w), w.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h
        p = C.c_int64()
        check(lib().hsc_mlp_n_params(self.h, C.byref(p)))
        self.n_params = int(p.value)

    def layout(self):
        """[(W offset, W shape, b offset, b size)] of the flat parameter vector."""
        out, o = [], 0
        for a, b in zip(self.widths[:-1], self.widths[1:]):
            out.append((o, (b, a), o + a * b, b))
            o += a * b + b
        return out

    def _f32(self, x, cols=None):
        import torch
        t = torch.as_tensor(x, dtype=torch.float32, device=self.ctx.torch_device).contiguous()
        if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
            raise ValueError(f"expected [n, {cols}] samples, got {tuple(t.shape)}")
        return t

    def set_params(self, params):
        p = self._f32(params).reshape(-1)
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        check(lib().hsc_mlp_set_params(self.ctx.h, self.h, _dptr(p)))
        self.ctx.sync()

    def get_params(self):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device=self.ctx.torch_device)
        check(lib().hsc_mlp_get_params(self.ctx.h, self.h, _dptr(p)))
        self.ctx.sync()
        return p

    def forward(self, x):
        import torch
        x = self._f32(x, self.widths[0])
        y = torch.empty((x.shape[0], self.widths[-1]), dtype=torch.float32, device=x.device)
        check(lib().hsc_mlp_forward(self.ctx.h, self.h, x.shape[0], _dptr(x), _dptr(y)))
        self.ctx.sync()
        return y

    def grads(self, x, t):
        import torch
        x, t = self._f32(x, self.widths[0]), self._f32(t, self.widths[-1])
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        check(lib().hsc_mlp_grads(self.ctx.h, self.h, x.shape[0], _dptr(x), _dptr(t), _dptr(g), _dptr(loss)))
        self.ctx.sync()
        return g, float(loss.item())

    def train(self, x, t, steps, lr=1e-3, batch=None, order=None, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam steps; order: int32 [steps * batch] sample indices (None = full batch). Returns the losses."""
        import torch
        x, t = self._f32(x, self.widths[0]), self._f32(t, self.widths[-1])
        n = x.shape[0]
        if order is not None:
            order = torch.as_tensor(order, dtype=torch.int32, device=x.device).contiguous()
            if batch is None or order.numel() != steps * batch:
                raise ValueError("order must hold steps * batch indices")
        hist = torch.empty(max(steps, 1), dtype=torch.float32, device=x.device)
        o = TrainOpts(lr, beta1, beta2, eps, int(batch or n), int(steps))
        check(lib().hsc_mlp_train(self.ctx.h, self.h, n, _dptr(x), _dptr(t), C.byref(o), _dptr(order), _dptr(hist)))
        self.ctx.sync()
        return hist[:steps].cpu().numpy()

    def close(self):
        if getattr(self, "h", None):
            lib().hsc_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
