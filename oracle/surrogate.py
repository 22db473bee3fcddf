"""FP64 oracle of the learned surrogate: an MLP that maps a kernel's
standardised baseline feature vector to the composed log-speedups of all 2^B
optimisation subsets in one pass.  The paper has no such network; it is an
extension trained on tables that the plain method (Tiers 1-3) produces, and
the plain method stays its fallback and judge.

Test infrastructure only (see the package docstring).

Network (row-vector convention, W of shape [fan_in, fan_out]):
  a1 = x W1 + b1,  h1 = gelu(a1)
  a2 = h1 W2 + b2, h2 = gelu(a2)
  y  = h2 W3 + b3
gelu(t) = t * Phi(t) = t/2 * (1 + erf(t / sqrt 2)) (exact form, not tanh).
Loss: mean over batch and outputs of (y - target)^2.
Adam (Kingma and Ba, 2015) with bias correction on FP64 master weights.
Initialisation: weights and biases U(-1/sqrt(fan_in), 1/sqrt(fan_in)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(t):
    return 0.5 * t * (1.0 + erf(t / SQRT2))


def gelu_grad(t):
    """d/dt [t Phi(t)] = Phi(t) + t phi(t)."""
    return 0.5 * (1.0 + erf(t / SQRT2)) + t * INV_SQRT_2PI * np.exp(-0.5 * t * t)


def init_params(rng: np.random.Generator, sizes) -> list:
    """[(W1, b1), (W2, b2), ...] for consecutive layer sizes."""
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        bound = 1.0 / math.sqrt(fi)
        W = rng.uniform(-bound, bound, size=(fi, fo))
        b = rng.uniform(-bound, bound, size=fo)
        params.append((W, b))
    return params


def forward(params, x, round_hidden=None):
    """Returns (y, cache).  ``round_hidden`` (optional) is applied to each
    hidden activation after the nonlinearity, to mirror a network that stores
    its activations at reduced precision."""
    h = np.asarray(x, dtype=np.float64)
    cache = {"x": h, "a": [], "h": [h]}
    nl = len(params)
    for i, (W, b) in enumerate(params):
        a = h @ W + b
        if i == nl - 1:
            cache["y"] = a
            return a, cache
        cache["a"].append(a)
        h = gelu(a)
        if round_hidden is not None:
            h = round_hidden(h)
        cache["h"].append(h)
    raise ValueError("empty network")


def mse(y, target):
    """Loss and its gradient with respect to y."""
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dy):
    """Hand-derived gradients [(dW1, db1), ...] of a scalar loss whose
    gradient with respect to the output is ``dy``."""
    grads = [None] * len(params)
    g = dy
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        h_in = cache["h"][i]
        grads[i] = (h_in.T @ g, g.sum(axis=0))
        if i > 0:
            g = (g @ W.T) * gelu_grad(cache["a"][i - 1])
    return grads


def adam_init(params):
    return {"t": 0,
            "m": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params],
            "v": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]}


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction; returns the new parameters and
    updates the moment state in place."""
    state["t"] += 1
    t = state["t"]
    out = []
    for i, (layer, glayer) in enumerate(zip(params, grads)):
        new = []
        for j in range(2):
            p, g = layer[j], glayer[j]
            m = beta1 * state["m"][i][j] + (1 - beta1) * g
            v = beta2 * state["v"][i][j] + (1 - beta2) * g * g
            state["m"][i][j], state["v"][i][j] = m, v
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    bfloat16 keeps the top 16 bits of an IEEE binary32 value."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u | 0x400000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, x):
    """The same network evaluated in FP64 on bfloat16-rounded weights, input
    and hidden activations (biases kept at full precision)."""
    pr = [(bf16_round(W), np.asarray(b, dtype=np.float64)) for W, b in params]
    return forward(pr, bf16_round(x), round_hidden=bf16_round)
