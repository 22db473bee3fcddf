"""Serving: profiling queries answered by the learned surrogate, judged and,
where it disagrees, answered by the plain per-optimisation models (Section 2's
Tier 2 stays the reference; the surrogate is an accelerator in front of it).

Per query of K kernels with B optimisations each (one library call,
sugg_serve_query; all work on one stream, every step a libsugg kernel):
  1. z0 = standardised baseline counters of each kernel (Tier 1, baseline rows)
  2. the surrogate's table for all 2^B subsets, then its top-n above tau
  3. the threshold band: for a kernel whose list is shorter than n, the other
     subsets within ``band`` below tau (at most ``cap``; more: fall back)
  4. judge: the plain composed value of the listed and band subsets, reading
     only the versions on their chains; a kernel where some surrogate value
     differs from the plain one by more than ``tol`` (log-speedup) is flagged
  5. flagged kernels are re-scored by the plain path (masked fused kernel);
     the others keep the surrogate's list, scored with the plain values.
Queries whose B has no trained surrogate, and queries too small to amortise
the surrogate's extra launches (fewer than ``min_rows`` profiled versions in
all; the plain path answers them in one launch), take the plain path
entirely.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np
import torch

from . import plain as G


class Server:
    def __init__(self, ctx: G.Context, nets: dict, n: int = 3, tol: float = 0.1, budget_bytes: int = 8 << 30,
                 band: float = 0.1, cap: int = 16, min_rows: int = 0):
        self.ctx, self.nets, self.n, self.tol, self.budget = ctx, nets, n, tol, budget_bytes
        self.band, self.cap, self.min_rows = band, cap, min_rows
        for m in nets.values():   # the served parameters, packed once
            m.freeze()
        self.plans = {}
        self.fallbacks = torch.zeros((), dtype=torch.int64, device=ctx.device)
        self.kernels_total = 0
        self.kernels_plain = 0       # answered by the plain path by policy (no surrogate tried)

    def plan(self, B: int, K: int, E: int, D: int):
        key = (B, K, E, D)
        if key not in self.plans:
            self.plans[key] = G.Plan(self.ctx, np.full(K, B, np.int32), np.tile(np.arange(B, dtype=np.int32), K), E, D)
        return self.plans[key]

    @staticmethod
    def footprint(K: int, B: int, E: int) -> int:
        """Bytes a query holds on the device: its counters and cycles, the
        surrogate's table and activations, the outputs."""
        rows = K << B
        return rows * (E + 1) * 4 + K * (1 << B) * 4 + K * (E + 2 * 512) * 4 + K * 64 * 4

    def answer(self, plan, counters, cycles, out):
        """Suggestions of one query into out = {"idx", "score", "count"};
        returns the per-kernel fallback flags (device int32) or None when the
        plain path answered the whole query."""
        B = int(plan.nopts[0]) if plan.K else 0
        mlp = self.nets.get(B)
        self.kernels_total += plan.K
        if mlp is None or plan.K > mlp.max_batch or plan.N < self.min_rows:
            G.suggest(self.ctx, plan, counters, cycles, out=out)
            self.kernels_plain += plan.K
            return None
        flag = torch.empty(plan.K, dtype=torch.int32, device=self.ctx.device)
        G.serve_query(self.ctx, plan, mlp, counters, cycles, out, flag, tol=self.tol, band=self.band, cap=self.cap)
        self.fallbacks += flag.sum()
        return flag


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def run_loop(server: Server, queries, arrivals, plain_only: bool = False, log=None):
    """Real-time loop: queries become ready at their arrival times, wait in a
    FIFO, are admitted if their footprint fits the HBM budget (else rejected),
    and are answered one at a time on the current stream.  Returns latency
    statistics (seconds from arrival to suggestions on the host)."""
    lat = np.full(len(queries), np.nan)
    rejected = 0
    queue = deque()
    i, done = 0, 0
    t0 = time.perf_counter()
    nets = server.nets
    if plain_only:
        server.nets = {}
    try:
        while done + rejected < len(queries):
            now = time.perf_counter() - t0
            while i < len(queries) and arrivals[i] <= now:
                queue.append(i)
                i += 1
            if not queue:
                if i < len(queries):
                    while time.perf_counter() - t0 < arrivals[i]:
                        pass
                continue
            q = queue.popleft()
            plan, counters, cycles, out, fp = queries[q]
            if fp > server.budget:
                rejected += 1
                continue
            server.answer(plan, counters, cycles, out)
            torch.cuda.current_stream().synchronize()
            lat[q] = time.perf_counter() - t0 - arrivals[q]
            done += 1
    finally:
        server.nets = nets
    span = time.perf_counter() - t0
    ok = lat[np.isfinite(lat)]
    kernels = sum(queries[j][0].K for j in range(len(queries)) if np.isfinite(lat[j]))
    return {"queries": int(done), "rejected": int(rejected), "p50_ms": float(np.percentile(ok, 50) * 1e3),
            "p99_ms": float(np.percentile(ok, 99) * 1e3), "mean_ms": float(ok.mean() * 1e3),
            "span_s": span, "kernels_per_s": kernels / span}
