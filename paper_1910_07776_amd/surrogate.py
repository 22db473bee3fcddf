"""Python binding of the learned surrogate (argument marshalling only; the
forward, backward, loss and Adam all run in libsugg's HIP kernels).

The surrogate maps a kernel's standardised baseline counter vector (Tier 1
features of its unoptimised version, Section 2) to the composed log-speedup of
every optimisation subset, one pass for the whole table.  It is trained on
tables that the plain per-optimisation models produce, and the plain models
stay its fallback and judge (see serve.py).

    mlp = MLP(ctx, 128, 512, 64, max_batch=4096, seed=0)
    y = SurrogateFn.apply(x, mlp.params, mlp)      # autograd: hand-written backward
    loss = mlp.train_step(x, target, lr=1e-3)      # fused loss/backward/Adam
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _abi as A
from .plain import Context, _ptr, _stream


def init_params(in_: int, hidden: int, out: int, seed: int = 0) -> np.ndarray:
    """Flat FP32 parameters W1 [h x in], b1, W2 [h x h], b2, W3 [out x h], b3,
    weights and biases drawn U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5A11])))
    parts = []
    for fi, fo in ((in_, hidden), (hidden, hidden), (hidden, out)):
        b = 1.0 / math.sqrt(fi)
        parts.append(rng.uniform(-b, b, size=(fo, fi)).ravel())
        parts.append(rng.uniform(-b, b, size=fo))
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """Surrogate network: FP32 master parameters, Adam moments and the
    library's workspace (BF16 working weights, kept activations)."""

    def __init__(self, ctx: Context, in_: int = 128, hidden: int = 512, out: int = 64,
                 max_batch: int = 4096, seed: int = 0, params=None):
        self.ctx, self.in_, self.hidden, self.out, self.max_batch = ctx, in_, hidden, out, max_batch
        h = C.c_void_p()
        A.check(ctx.h, A.lib().sugg_mlp_create(ctx.h, in_, hidden, out, max_batch, C.byref(h)))
        self.h = h
        self.P = int(A.lib().sugg_mlp_param_count(h))
        p = init_params(in_, hidden, out, seed) if params is None else np.asarray(params, np.float32)
        if p.size != self.P:
            raise ValueError(f"expected {self.P} parameters, got {p.size}")
        dev = ctx.device
        self.params = torch.tensor(p, device=dev)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.loss = torch.zeros(1, device=dev)

    def close(self):
        if getattr(self, "h", None):
            A.lib().sugg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # layout of the flat parameter vector
    def shapes(self):
        i, h, o = self.in_, self.hidden, self.out
        return [("W1", (h, i)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (o, h)), ("b3", (o,))]

    def unflatten(self, flat):
        out, k = {}, 0
        for name, shp in self.shapes():
            n = int(np.prod(shp))
            out[name] = flat[k:k + n].reshape(shp)
            k += n
        return out

    def _check_x(self, x, width):
        if x.dtype != torch.float32 or not x.is_contiguous() or x.device != self.ctx.device or x.dim() != 2 \
                or x.shape[1] != width or not (1 <= x.shape[0] <= self.max_batch):
            raise ValueError(f"expected a contiguous float32 [batch <= {self.max_batch} x {width}] tensor on "
                             f"{self.ctx.device}")

    def forward_raw(self, params, x, keep=False, y=None):
        self._check_x(x, self.in_)
        B = x.shape[0]
        if y is None:
            y = torch.empty((B, self.out), device=self.ctx.device)
        A.check(self.ctx.h, A.lib().sugg_mlp_forward(self.ctx.h, self.h, _ptr(params), _ptr(x), B, _ptr(y),
                                                     int(keep), _stream()))
        return y

    def backward_raw(self, params, dy, B, grads):
        if dy is not None:
            self._check_x(dy, self.out)
        A.check(self.ctx.h, A.lib().sugg_mlp_backward(self.ctx.h, self.h, _ptr(params), _ptr(dy), B, _ptr(grads),
                                                      _stream()))
        return grads

    def __call__(self, x, y=None):
        return self.forward_raw(self.params, x, keep=False, y=y)

    def loss_raw(self, x, target, y=None):
        self._check_x(x, self.in_)
        self._check_x(target, self.out)
        A.check(self.ctx.h, A.lib().sugg_mlp_loss(self.ctx.h, self.h, _ptr(self.params), _ptr(x), _ptr(target),
                                                  x.shape[0], _ptr(y), _ptr(self.loss), _stream()))
        return self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        A.check(self.ctx.h, A.lib().sugg_mlp_adam(self.ctx.h, self.h, _ptr(self.params), _ptr(self.grads),
                                                  _ptr(self.m), _ptr(self.v), self.step, lr, beta1, beta2, eps,
                                                  _stream()))

    def train_step(self, x, target, lr=1e-3):
        """Loss, backward and Adam in one call; returns the device loss."""
        self._check_x(x, self.in_)
        self._check_x(target, self.out)
        self.step += 1
        A.check(self.ctx.h, A.lib().sugg_mlp_train_step(self.ctx.h, self.h, _ptr(self.params), _ptr(self.grads),
                                                        _ptr(self.m), _ptr(self.v), self.step, lr, _ptr(x),
                                                        _ptr(target), x.shape[0], _ptr(self.loss), _stream()))
        return self.loss

    def state_dict(self):
        return {"params": self.params.clone(), "m": self.m.clone(), "v": self.v.clone(), "step": self.step,
                "shape": (self.in_, self.hidden, self.out)}

    def load_state_dict(self, sd):
        if tuple(sd["shape"]) != (self.in_, self.hidden, self.out):
            raise ValueError("shape mismatch")
        self.params.copy_(sd["params"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step = int(sd["step"])


class SurrogateFn(torch.autograd.Function):
    """y = MLP(x; params) with the library's hand-written backward.  One
    forward may be outstanding per MLP object (its kept activations)."""

    @staticmethod
    def forward(fctx, x, params, mlp):
        y = mlp.forward_raw(params.detach(), x.detach().contiguous(), keep=True)
        fctx.mlp = mlp
        fctx.B = x.shape[0]
        fctx.save_for_backward(params)
        return y

    @staticmethod
    def backward(fctx, dy):
        (params,) = fctx.saved_tensors
        grads = torch.empty_like(params)
        fctx.mlp.backward_raw(params.detach(), dy.contiguous().float(), fctx.B, grads)
        return None, grads, None
