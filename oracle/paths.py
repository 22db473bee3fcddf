"""FP64 oracle of two uses of the single-optimisation predictions beyond the
ascending-chain composition.  Test infrastructure only (see the package
docstring).

All-paths composition.  The paper predicts the benefit of adding one
optimisation to one profiled version (Section 2, Tier 2); it does not say how
to score a set of several.  Adding the optimisations of S one at a time along
any order gives an estimate; the all-paths estimate averages over every
order, which removes the arbitrary choice of one chain:
    L(0) = 0,   L(S) = (1/|S|) * sum over b in S of [ L(S - b) + P(S - b, b) ],
the mean over the |S|! orderings of S of the predictions summed along it
(each b is the last of (|S|-1)! of them).

Greedy re-profiling.  The tool is meant to be used iteratively (Section 2:
the user applies a suggested optimisation, profiles the new version and asks
again).  Simulated on a kernel whose every version has been profiled: start
from the baseline S = 0; while some optimisation b not in S has a predicted
benefit P(S, b) above the threshold, apply the best one (ties: the smaller
bit) and continue from the profiled version S + b.
"""
from __future__ import annotations

import itertools

import numpy as np

from .plain import N_SUGGEST, TAU, rank


def popcount(S: int) -> int:
    return bin(S).count("1")


def compose_allpaths(grid: np.ndarray, batch) -> np.ndarray:
    """All-paths composed log-speedups [N] from the single-optimisation grid
    (grid[row(k, S), b] = P(S, b) for b not in S), level by level in |S|."""
    table = np.zeros(grid.shape[0])
    for k in range(len(batch.nopts)):
        B, r0 = int(batch.nopts[k]), int(batch.row_off[k])
        L = np.zeros(1 << B)
        for S in sorted(range(1, 1 << B), key=popcount):
            terms = [L[S & ~(1 << b)] + grid[r0 + (S & ~(1 << b)), b] for b in range(B) if (S >> b) & 1]
            L[S] = sum(terms) / len(terms)
        table[r0:r0 + (1 << B)] = L
    return table


def allpaths_by_orderings(P: np.ndarray, S: int) -> float:
    """The same quantity for one kernel's grid P [2^B, B] by brute force:
    the mean over every ordering of S of the predictions summed along it."""
    bits = [b for b in range(P.shape[1]) if (S >> b) & 1]
    if not bits:
        return 0.0
    total, count = 0.0, 0
    for order in itertools.permutations(bits):
        cur, acc = 0, 0.0
        for b in order:
            acc += P[cur, b]
            cur |= 1 << b
        total += acc
        count += 1
    return total / count


def greedy_kernel(P: np.ndarray, B: int, tau: float = TAU):
    """Greedy re-profiling on one kernel's grid P [2^B, B]: the visited
    versions (starting with 0) and the predicted log-speedups of the steps."""
    S, path, steps = 0, [0], []
    while True:
        cand = np.full(B, -np.inf)
        for b in range(B):
            if not (S >> b) & 1:
                cand[b] = P[S, b]
        best = rank(cand, tau, 1)
        if not best:
            return path, steps
        b, v = best[0]
        S |= 1 << b
        path.append(S)
        steps.append(v)


def greedy(grid: np.ndarray, batch, tau: float = TAU):
    """greedy_kernel for every kernel of a batch."""
    out = []
    for k in range(len(batch.nopts)):
        B, r0 = int(batch.nopts[k]), int(batch.row_off[k])
        out.append(greedy_kernel(grid[r0:r0 + (1 << B), :B], B, tau))
    return out


def suggest_allpaths(grid: np.ndarray, batch, tau: float = TAU, n: int = N_SUGGEST):
    """Top-n subsets per kernel of the all-paths table (Tier 3's ranking)."""
    table = compose_allpaths(grid, batch)
    res = []
    for k in range(len(batch.nopts)):
        r0, r1 = int(batch.row_off[k]), int(batch.row_off[k + 1])
        res.append(rank(table[r0:r1], tau, n, first=1))
    return table, res
