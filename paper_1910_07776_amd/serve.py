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

Admission (run_loop): up to four queries in flight, one per stream slot of
default priority, while the device bytes they hold stay within the HBM
budget; a query larger than the whole budget is rejected.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np
import torch

from . import plain as G


class Server:
    """Answers queries on ``streams`` (1-4) CUDA streams of default priority;
    each stream slot has its own plans and its own copy of every surrogate
    (workspace), so queries on different slots run concurrently."""

    def __init__(self, ctx: G.Context, nets: dict, n: int = 3, tol: float = 0.1, budget_bytes: int = 8 << 30,
                 band: float = 0.1, cap: int = 16, min_rows: int = 0, streams: int = 1):
        if not 1 <= streams <= 4:
            raise ValueError("streams must be 1..4")
        self.ctx, self.nets, self.n, self.tol, self.budget = ctx, nets, n, tol, budget_bytes
        self.band, self.cap, self.min_rows = band, cap, min_rows
        for m in nets.values():   # the served parameters, packed once
            m.freeze()
        self.streams = [torch.cuda.current_stream(ctx.device)] if streams == 1 else \
            [torch.cuda.Stream(ctx.device) for _ in range(streams)]
        self.slot_nets = [nets] + [{B: self._copy(m) for B, m in nets.items()} for _ in range(1, streams)]
        self.plans = {}
        self.slot_fallbacks = [torch.zeros((), dtype=torch.int64, device=ctx.device) for _ in range(streams)]
        self.kernels_total = 0
        self.kernels_plain = 0       # answered by the plain path by policy (no surrogate tried)
        self.plain_only = False

    def _copy(self, m):
        from .surrogate import MLP
        c = MLP(self.ctx, m.in_, m.hidden, m.out, max_batch=m.max_batch, params=m.params.detach().cpu().numpy())
        return c.freeze()

    def close(self):
        for nets in self.slot_nets[1:]:
            for m in nets.values():
                m.close()
        self.slot_nets = self.slot_nets[:1]

    def prepare(self, queries):
        """Builds every slot's plans and workspaces for these queries (one
        untimed answer of each distinct query shape on every slot)."""
        seen = set()
        for plan, counters, cycles, out, _ in queries:
            key = (int(plan.nopts[0]) if plan.K else 0, plan.K, plan.E, plan.D)
            if key in seen:
                continue
            seen.add(key)
            for slot, st in enumerate(self.streams):
                with torch.cuda.stream(st):
                    self.answer(plan, counters, cycles, out, slot)
        for st in self.streams:
            st.synchronize()
        self.reset_counts()

    @property
    def fallbacks(self):
        return sum(self.slot_fallbacks)

    def reset_counts(self):
        for f in self.slot_fallbacks:
            f.zero_()
        self.kernels_total = self.kernels_plain = 0

    def plan(self, B: int, K: int, E: int, D: int, slot: int = 0):
        key = (slot, B, K, E, D)
        if key not in self.plans:
            self.plans[key] = G.Plan(self.ctx, np.full(K, B, np.int32), np.tile(np.arange(B, dtype=np.int32), K), E, D)
        return self.plans[key]

    @staticmethod
    def footprint(K: int, B: int, E: int) -> int:
        """Bytes a query holds on the device: its counters and cycles, the
        surrogate's table and activations, the outputs."""
        rows = K << B
        return rows * (E + 1) * 4 + K * (1 << B) * 4 + K * (E + 2 * 512) * 4 + K * 64 * 4

    def answer(self, plan, counters, cycles, out, slot: int = 0):
        """Suggestions of one query into out = {"idx", "score", "count"} on
        the current stream, with the slot's plans and surrogates; returns the
        per-kernel fallback flags (device int32) or None when the plain path
        answered the whole query."""
        B = int(plan.nopts[0]) if plan.K else 0
        if slot:
            plan = self.plan(B, plan.K, plan.E, plan.D, slot)
        mlp = None if self.plain_only else self.slot_nets[slot].get(B)
        self.kernels_total += plan.K
        if mlp is None or plan.K > mlp.max_batch or plan.N < self.min_rows:
            G.suggest(self.ctx, plan, counters, cycles, out=out)
            self.kernels_plain += plan.K
            return None
        flag = torch.empty(plan.K, dtype=torch.int32, device=self.ctx.device)
        G.serve_query(self.ctx, plan, mlp, counters, cycles, out, flag, tol=self.tol, band=self.band, cap=self.cap)
        self.slot_fallbacks[slot] += flag.sum()
        return flag


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def run_loop(server: Server, queries, arrivals, plain_only: bool = False, log=None):
    """Real-time loop: queries become ready at their arrival times and wait in
    a FIFO.  The head is rejected if its footprint alone exceeds the HBM
    budget; otherwise it is admitted once a stream slot is free and the
    footprints of the queries in flight plus its own fit the budget (until
    then it and everything behind it wait).  A query's latency runs from its
    arrival to the host seeing its stream's completion event.  Returns latency
    and admission statistics."""
    lat = np.full(len(queries), np.nan)
    rejected, waited = 0, 0
    queue = deque()
    inflight = []                     # (query, slot, event, bytes)
    free = list(range(len(server.streams)))[::-1]
    used = max_used = max_q = 0
    head_waited = -1
    i, done = 0, 0
    t0 = time.perf_counter()
    server.plain_only = plain_only
    try:
        while done + rejected < len(queries):
            now = time.perf_counter() - t0
            while i < len(queries) and arrivals[i] <= now:
                queue.append(i)
                i += 1
            for e in [e for e in inflight if e[2].query()]:
                lat[e[0]] = time.perf_counter() - t0 - arrivals[e[0]]
                used -= e[3]
                free.append(e[1])
                inflight.remove(e)
                done += 1
            while queue:
                q = queue[0]
                plan, counters, cycles, out, fp = queries[q]
                if fp > server.budget:
                    queue.popleft()
                    rejected += 1
                    continue
                if not free or used + fp > server.budget:
                    if head_waited != q:
                        waited += 1
                        head_waited = q
                    break
                queue.popleft()
                slot = free.pop()
                st = server.streams[slot]
                with torch.cuda.stream(st):
                    server.answer(plan, counters, cycles, out, slot)
                ev = torch.cuda.Event()
                ev.record(st)
                inflight.append((q, slot, ev, fp))
                used += fp
                max_used, max_q = max(max_used, used), max(max_q, len(inflight))
            if not queue and not inflight and i < len(queries):
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
    finally:
        server.plain_only = False
    for st in server.streams:
        st.synchronize()
    span = time.perf_counter() - t0
    ok = lat[np.isfinite(lat)]
    kernels = sum(queries[j][0].K for j in range(len(queries)) if np.isfinite(lat[j]))
    return {"queries": int(done), "rejected": int(rejected), "waited_for_admission": int(waited),
            "max_in_flight": int(max_q), "max_in_flight_bytes": int(max_used), "budget_bytes": int(server.budget),
            "streams": len(server.streams),
            "p50_ms": float(np.percentile(ok, 50) * 1e3) if ok.size else None,
            "p99_ms": float(np.percentile(ok, 99) * 1e3) if ok.size else None,
            "mean_ms": float(ok.mean() * 1e3) if ok.size else None,
            "span_s": span, "kernels_per_s": kernels / span}


def plain_agreement(server: Server, queries) -> dict:
    """How often the served answers equal the plain path's top-n (same
    subsets in the same order), over every kernel of the queries; run after a
    loop, on slot 0 (not timed)."""
    same = total = same_set = 0
    for plan, counters, cycles, out, _ in queries:
        ref = G.suggest(server.ctx, plan, counters, cycles, table=False)
        ci, cc = out["idx"], out["count"]
        eq = (ci == ref[0]).all(dim=1) & (cc == ref[2])
        same += int(eq.sum())
        a, _ = torch.sort(torch.where(ci >= 0, ci, 1 << 20), dim=1)
        b, _ = torch.sort(torch.where(ref[0] >= 0, ref[0], 1 << 20), dim=1)
        same_set += int(((a == b).all(dim=1) & (cc == ref[2])).sum())
        total += plan.K
    return {"kernels": total, "same_list": same / max(1, total), "same_set": same_set / max(1, total)}
