"""The same synthetic world drawn on the GPU with torch, for training sets too
large to draw on the host (a million kernels x 64 versions x 128 events).

World parameters (mu, bias, w, gamma, delta) are the NumPy world's
(``world.world_for``); the per-kernel draws (a, eps, eta) come from a torch
generator on the device seeded per chunk, so a chunk is reproducible on one
device but is a different draw than ``make_batch`` of the same ids.  Every
kernel has all D optimisations (B = D), as in the 6-optimisation lattices of
Section 3.3 (or the first B of them).  Input generation only: no part of the
suggestion method.
"""
from __future__ import annotations

import math

import torch

from .world import COUNTER_SIGMA, EPS_SIGMA, ETA_SIGMA, world_for


def _chunk_seed(seed: int, chunk: int) -> int:
    return (int(seed) * 1_000_003 + int(chunk) * 7_919 + 0x5EED) % (2 ** 62)


class TorchWorld:
    def __init__(self, seed: int, E: int, D: int, device="cuda", B: int | None = None):
        wd = world_for(seed, E, D)
        B = D if B is None else int(B)
        if not 0 <= B <= D:
            raise ValueError("B must be in [0, D]")
        self.seed, self.E, self.D, self.B = seed, E, D, B
        f = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)  # noqa: E731
        # kernels carry the first B of the D global optimisations
        self.mu, self.bias, self.w = f(wd.mu), f(wd.bias[:B]), f(wd.w[:B])
        self.gamma, self.delta = f(wd.gamma[:B, :B]), f(wd.delta[:B])
        n = 1 << B
        S = torch.arange(n, device=device)
        self.bits = ((S[:, None] >> torch.arange(B, device=device)) & 1).to(torch.float64)   # [n, B]
        self.pair = 0.5 * ((self.bits @ self.gamma) * self.bits).sum(1)                    # [n]
        self.shift = self.bits @ self.delta                                                # [n, E]
        self.device = device

    def chunk(self, chunk: int, K: int, dtype=torch.float32):
        """Kernels of chunk ``chunk``: counters [K*2^B, E], cycles [K*2^B] and
        the true log-speedups [K, 2^B] (rows kernel after kernel, version S at
        kernel offset S)."""
        g = torch.Generator(device=self.device)
        g.manual_seed(_chunk_seed(self.seed * 64 + self.B, chunk))
        E, n = self.E, 1 << self.B
        a = torch.randn((K, E + 1), generator=g, device=self.device, dtype=torch.float64)
        lc0 = self.mu + COUNTER_SIGMA * a
        u = (a[:, :E] - a[:, E:]) / math.sqrt(2.0)
        lin = u @ self.w.T + self.bias                                 # [K, D]
        T = lin @ self.bits.T + self.pair                              # [K, n]
        eps = EPS_SIGMA * torch.randn((K, n - 1), generator=g, device=self.device, dtype=torch.float64)
        T[:, 1:] += eps
        eta = torch.randn((K, n, E), generator=g, device=self.device, dtype=dtype)
        eta.mul_(ETA_SIGMA)
        eta += (lc0[:, None, :E] + self.shift[None]).to(dtype)
        counters = eta.exp_().reshape(K * n, E)
        cycles = torch.exp(lc0[:, E:] - T).to(dtype).reshape(K * n)
        return counters, cycles, T
