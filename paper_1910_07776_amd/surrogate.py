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

    def freeze(self, params=None):
        """Keep a copy of the parameters (default: the current ones) for
        serving queries (``plain.serve_query``)."""
        p = self.params if params is None else params
        A.check(self.ctx.h, A.lib().sugg_mlp_freeze(self.ctx.h, self.h, _ptr(p), _stream()))
        return self

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

    def infer(self, x, y=None):
        """Inference with the frozen parameters (``freeze`` first)."""
        self._check_x(x, self.in_)
        if y is None:
            y = torch.empty((x.shape[0], self.out), device=self.ctx.device)
        A.check(self.ctx.h, A.lib().sugg_mlp_infer(self.ctx.h, self.h, _ptr(x), x.shape[0], _ptr(y), _stream()))
        return y

    def infer_rank(self, x, n: int = 3, tau: float = 0.0, skip: int = 1, y=None, out=None):
        """Inference with the frozen parameters and each row's top n outputs
        above tau (columns >= skip): returns (idx, score, count), written into
        ``out`` when given; the outputs themselves into y when given."""
        self._check_x(x, self.in_)
        B = x.shape[0]
        if out is None:
            out = (torch.empty((B, n), dtype=torch.int32, device=self.ctx.device),
                   torch.empty((B, n), device=self.ctx.device),
                   torch.empty(B, dtype=torch.int32, device=self.ctx.device))
        idx, sc, cnt = out
        A.check(self.ctx.h, A.lib().sugg_mlp_infer_rank(self.ctx.h, self.h, _ptr(x), B, skip, n, float(tau), _ptr(y),
                                                        _ptr(idx), _ptr(sc), _ptr(cnt), _stream()))
        return idx, sc, cnt

    def train_epoch(self, X, Y, perm, batch: int, lr=1e-3):
        """len(perm) // batch training steps in one library call over the
        mini-batches X[perm[s*batch:(s+1)*batch]] (gathered on the device);
        returns the per-step losses (device)."""
        self._check_x(X[:1], self.in_)
        self._check_x(Y[:1], self.out)
        if not (X.is_contiguous() and Y.is_contiguous() and X.shape[0] == Y.shape[0]):
            raise ValueError("X and Y must be contiguous with one row per sample")
        if perm.dtype != torch.int32 or not perm.is_contiguous() or perm.device != self.ctx.device:
            raise ValueError("perm must be a contiguous int32 tensor on the device")
        if not 1 <= batch <= self.max_batch:
            raise ValueError(f"batch outside [1, {self.max_batch}]")
        steps = perm.numel() // batch
        losses = torch.zeros(steps, device=self.ctx.device)
        A.check(self.ctx.h, A.lib().sugg_mlp_train_epoch(
            self.ctx.h, self.h, _ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v), self.step, lr,
            _ptr(X), _ptr(Y), X.shape[0], _ptr(perm), batch, steps, _ptr(losses), _stream()))
        self.step += steps
        return losses

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


# ---------------------------------------------------------------- training --
def label_chunk(ctx, plan, counters, cycles, B: int, with_baseline_grid: bool = False):
    """Plain-method labels of a uniform batch (every kernel B optimisations):
    X = standardised baseline counters [K, E], Y = composed tables [K, 2^B]
    (sugg_predict), and optionally the grid's baseline rows [K, B] (the plain
    models' single-optimisation predictions P(baseline, b))."""
    from .plain import load_features, predict
    table, grid = predict(ctx, plan, counters, cycles, grid=with_baseline_grid)
    X = load_features(ctx, plan, counters, cycles, baseline=True)
    Y = table.view(plan.K, 1 << B)
    g0 = None
    if with_baseline_grid:
        g0 = grid[torch.as_tensor(plan.row_off[:-1], device=grid.device)][:, :B]
    return X, Y, g0


def build_dataset(ctx, tw, n_kernels: int, chunk: int = 65536, chunk_base: int = 0, with_truth: bool = False,
                  with_baseline_grid: bool = False):
    """Draw n_kernels kernels of the TorchWorld tw in chunks and label them
    with the plain path.  Returns a dict of device tensors X, Y (and T, the
    generator's true log-speedups; G0, the grid's baseline rows)."""
    from .plain import Plan
    B, E, dev = tw.B, tw.E, ctx.device
    out = {"X": torch.empty((n_kernels, E), device=dev), "Y": torch.empty((n_kernels, 1 << B), device=dev)}
    if with_truth:
        out["T"] = torch.empty((n_kernels, 1 << B), device=dev)
    if with_baseline_grid:
        out["G0"] = torch.empty((n_kernels, B), device=dev)
    plans = {}
    for i, c0 in enumerate(range(0, n_kernels, chunk)):
        K = min(chunk, n_kernels - c0)
        if K not in plans:
            plans[K] = Plan(ctx, np.full(K, B, np.int32), np.tile(np.arange(B, dtype=np.int32), K), E, tw.D)
        counters, cycles, truth = tw.chunk(chunk_base + i, K)
        X, Y, g0 = label_chunk(ctx, plans[K], counters, cycles, B, with_baseline_grid)
        out["X"][c0:c0 + K] = X
        out["Y"][c0:c0 + K] = Y
        if with_truth:
            out["T"][c0:c0 + K] = truth.float()
        if with_baseline_grid:
            out["G0"][c0:c0 + K] = g0
        del counters, cycles
    return out


def predict_table(mlp: MLP, X: torch.Tensor, batch: int | None = None) -> torch.Tensor:
    """Surrogate table for every row of X, in batches of the MLP's capacity."""
    batch = batch or mlp.max_batch
    Y = torch.empty((X.shape[0], mlp.out), device=X.device)
    for i in range(0, X.shape[0], batch):
        mlp(X[i:i + batch].contiguous(), y=Y[i:i + batch])
    return Y


def mape(pred: torch.Tensor, truth: torch.Tensor) -> float:
    """Mean absolute percentage error of predicted speedups e^pred against
    e^truth over every kernel and subset S != 0 (column 0 is the baseline)."""
    p, t = pred[:, 1:].double(), truth[:, 1:].double()
    return float((torch.abs(torch.exp(p) - torch.exp(t)) / torch.exp(t)).mean().item())


def train(mlp: MLP, X: torch.Tensor, Y: torch.Tensor, epochs: int, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, val=None, target_mape=None, check_every: int = 5, log=None):
    """Adam on the MSE of log-speedups over shuffled mini-batches.  Stops early
    once val = (X, T) gives a MAPE <= target_mape.  Returns a history list."""
    dev = X.device
    n = X.shape[0]
    steps = max(1, n // batch)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    hist = []
    for ep in range(1, epochs + 1):
        perm = torch.randperm(n, generator=g, device=dev)[:steps * batch].to(torch.int32)
        losses = mlp.train_epoch(X, Y, perm, batch, lr)
        rec = {"epoch": ep, "loss": float(losses.sum().item()) / steps}
        if val is not None and (ep % check_every == 0 or ep == epochs):
            rec["val_mape"] = mape(predict_table(mlp, val[0]), val[1])
        hist.append(rec)
        if log:
            log(rec)
        if target_mape is not None and rec.get("val_mape", 1e9) <= target_mape:
            break
    return hist
