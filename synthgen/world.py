"""Seeded synthetic counter worlds.

The paper profiles every version of a program built from all subsets of its
binary optimizations (Section 3.3: six optimizations, 64 versions, 32 with and
32 without each) and feeds per-run hardware counters plus the cycle count to
its tool (Section 2, Tier 1; three runs per version, Section 5).  None of that
data exists here, so this module draws a synthetic world with the same shape:

World (seed ``ws``; ``Generator(PCG64(SeedSequence([ws])))``, draw order fixed)
  mu[j]      ~ U[2, 12]            j = 0..E   (index E is the cycle count)
  bias[o]    ~ U[-0.05, 0.20]      o = 0..D-1
  w[o, j]    ~ N(0, 0.15^2 / E)    per-optimisation linear term
  gamma[o,p] ~ N(0, 0.03^2)        pairwise interaction, symmetric, o < p drawn
  delta[o,j] ~ N(0, 0.1^2)         the optimisation's effect on the counters

Kernel k (seed ``SeedSequence([ws, k])``, regenerable on its own)
  B_k, O_k   fixed (B = D, O = 0..D-1) or B ~ U{Bmin..Bmax}, O = sorted subset
  a[j]       ~ N(0, 1)             j = 0..E
  ln c0[j]   = mu[j] + 0.5 a[j]    (lognormal counters, sigma 0.5)
  u[j]       = (a[j] - a[E]) / sqrt(2)       analytic standardised log-rate
  T[S]       = sum_{b in S} (w[O_b] . u + bias[O_b])
               + sum_{b < b' in S} gamma[O_b, O_b'] + eps_S
  eps_S      ~ N(0, 0.05^2) for S >= 1, eps_0 = 0
  eta[S, j]  ~ N(0, 0.02^2)        per-run counter jitter
  ln c[S, j] = ln c0[j] + sum_{b in S} delta[O_b, j] + eta[S, j]
               (eta is drawn in the batch dtype and exp'd in that dtype)
  ln cyc[S]  = ln c0[E] - T[S]     so T[S] is the true log-speedup of version S

Rows of kernel k sit at ``row_off[k] + S`` where S is the subset bitmask over
the kernel's local optimisation bits (bit b <-> global id O_k[b]).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
from threadpoolctl import threadpool_limits

COUNTER_SIGMA = 0.5
EPS_SIGMA = 0.05
ETA_SIGMA = 0.02
W_SD = 0.15
GAMMA_SD = 0.03
DELTA_SD = 0.1


def _rng(*words: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(words))))


@dataclass(frozen=True)
class World:
    seed: int
    E: int
    D: int
    mu: np.ndarray       # [E+1]
    bias: np.ndarray     # [D]
    w: np.ndarray        # [D, E]
    gamma: np.ndarray    # [D, D] symmetric, zero diagonal
    delta: np.ndarray    # [D, E]


_WORLDS: dict = {}


def world_for(seed: int, E: int, D: int) -> World:
    key = (int(seed), int(E), int(D))
    if key in _WORLDS:
        return _WORLDS[key]
    rng = _rng(seed)
    mu = rng.uniform(2.0, 12.0, size=E + 1)
    bias = rng.uniform(-0.05, 0.20, size=D)
    w = rng.normal(0.0, W_SD / np.sqrt(E), size=(D, E))
    g = rng.normal(0.0, GAMMA_SD, size=(D, D))
    g = np.triu(g, 1)
    gamma = g + g.T
    delta = rng.normal(0.0, DELTA_SD, size=(D, E))
    wd = World(int(seed), int(E), int(D), mu, bias, w, gamma, delta)
    _WORLDS[key] = wd
    return wd


@dataclass
class Batch:
    """A ragged batch of profiled kernels, each with all 2^B_k versions."""
    K: int
    E: int
    D: int
    dtype: np.dtype
    kernel_ids: np.ndarray   # [K] int64 (generator ids)
    nopts: np.ndarray        # [K] int32, B_k
    opt_ids: np.ndarray      # [sum B_k] int32, ascending within a kernel
    opt_off: np.ndarray      # [K+1] int64
    row_off: np.ndarray      # [K+1] int64, row_off[k+1]-row_off[k] = 2^B_k
    counters: np.ndarray     # [N, E] dtype
    cycles: np.ndarray       # [N] dtype
    truth: np.ndarray        # [N] float64, T[S] of each row (T[0] = 0)
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.row_off[-1])

    def kernel_opts(self, k: int) -> np.ndarray:
        return self.opt_ids[self.opt_off[k]:self.opt_off[k + 1]]

    def kernel_rows(self, k: int) -> slice:
        return slice(int(self.row_off[k]), int(self.row_off[k + 1]))


def kernel_layout(nopts: np.ndarray):
    """Row and option offsets of a ragged batch (prefix sums of 2^B_k and B_k)."""
    nopts = np.asarray(nopts, dtype=np.int64)
    row_off = np.zeros(len(nopts) + 1, dtype=np.int64)
    np.cumsum(np.left_shift(1, nopts), out=row_off[1:])
    opt_off = np.zeros(len(nopts) + 1, dtype=np.int64)
    np.cumsum(nopts, out=opt_off[1:])
    return row_off, opt_off


def _kernel_structure(wd: World, k: int, brange):
    rng = _rng(wd.seed, k)
    if brange is None:
        B = wd.D
        O = np.arange(wd.D, dtype=np.int64)
    else:
        lo, hi = brange
        B = int(rng.integers(lo, hi + 1))
        O = np.sort(rng.choice(wd.D, size=B, replace=False)).astype(np.int64)
    return rng, B, O


def _draw_kernel(wd: World, rng, B: int, O: np.ndarray, out_c, out_cyc, out_t):
    E = wd.E
    a = rng.standard_normal(E + 1)
    lc0 = wd.mu + COUNTER_SIGMA * a
    u = (a[:E] - a[E]) / np.sqrt(2.0)
    n = 1 << B
    eps = rng.normal(0.0, EPS_SIGMA, size=n - 1)
    S = np.arange(n, dtype=np.int64)
    bits = ((S[:, None] >> np.arange(B)) & 1).astype(np.float64)       # [n, B]
    lin = wd.w[O] @ u + wd.bias[O]                                      # [B]
    g = wd.gamma[np.ix_(O, O)]                                          # zero diagonal
    T = bits @ lin + 0.5 * ((bits @ g) * bits).sum(axis=1)
    T[1:] += eps
    # per-run jitter drawn straight into the output rows, in the output dtype
    rng.standard_normal(out=out_c, dtype=out_c.dtype)
    out_c *= ETA_SIGMA
    out_c += (lc0[:E] + bits @ wd.delta[O]).astype(out_c.dtype)
    np.exp(out_c, out=out_c)
    out_cyc[...] = np.exp(lc0[E] - T)
    out_t[...] = T


def make_batch(seed: int, kernel_ids, E: int, D: int, brange=None,
               dtype=np.float32, threads: int | None = None) -> Batch:
    """Draw kernels ``kernel_ids`` of world (seed, E, D).

    ``brange=None`` gives every kernel all D optimisations (B = D); otherwise
    ``brange=(Bmin, Bmax)`` draws B_k uniformly and a sorted random subset of
    the D global optimisation ids.
    """
    wd = world_for(seed, E, D)
    kid = np.asarray(list(kernel_ids), dtype=np.int64)
    K = len(kid)
    structs = [_kernel_structure(wd, int(k), brange) for k in kid]
    nopts = np.array([s[1] for s in structs], dtype=np.int32)
    row_off, opt_off = kernel_layout(nopts)
    opt_ids = (np.concatenate([s[2] for s in structs]).astype(np.int32)
               if K else np.zeros(0, np.int32))
    N = int(row_off[-1])
    dt = np.dtype(dtype)
    counters = np.empty((N, E), dtype=dt)
    cycles = np.empty(N, dtype=dt)
    truth = np.empty(N, dtype=np.float64)

    def work(ks):
        for i in ks:
            rng, B, O = structs[i]
            r0, r1 = int(row_off[i]), int(row_off[i + 1])
            _draw_kernel(wd, rng, B, O, counters[r0:r1], cycles[r0:r1], truth[r0:r1])

    nt = threads if threads is not None else min(16, os.cpu_count() or 1)
    # the per-kernel products are tiny: keep BLAS single-threaded so the
    # kernel-level thread pool is not oversubscribed
    with threadpool_limits(limits=1, user_api="blas"):
        if N * E < 2_000_000 or nt <= 1:
            work(range(K))
        else:
            chunks = np.array_split(np.arange(K), nt * 4)
            with ThreadPoolExecutor(nt) as ex:
                list(ex.map(work, chunks))
    return Batch(K, E, D, dt, kid, nopts, opt_ids, opt_off, row_off,
                 counters, cycles, truth)
