"""Tolerance-aware checks of suggestion lists against the FP64 oracle.

Test infrastructure only.  When two candidates' oracle scores differ by less
than the comparison tolerance, either order is a correct answer; the same holds
for a candidate within the tolerance of the threshold or of the n-th place.
Everything else (which subsets, how many, their order) must match exactly.
"""
from __future__ import annotations

import numpy as np


def check_list(got_idx, got_score, ora_scores, tau: float, n: int, tol: float,
               first: int = 0, score_rtol: float | None = None) -> list[str]:
    """Return a list of problems (empty when ``got`` is a correct top-n list).

    got_idx     indices chosen by the implementation under test, best first
    got_score   their scores as computed by that implementation
    ora_scores  the oracle's scores of every index of the segment (FP64)
    tol         absolute tolerance on a score (log-speedup)
    score_rtol  tolerance on e^score of each reported score (default: tol)
    """
    s = np.asarray(ora_scores, dtype=np.float64)
    idx = [int(i) for i in got_idx]
    errs = []
    rt = tol if score_rtol is None else score_rtol
    if len(idx) > n:
        errs.append(f"{len(idx)} entries > n={n}")
    if len(set(idx)) != len(idx):
        errs.append(f"duplicate indices {idx}")
    for i in idx:
        if not (first <= i < len(s)):
            errs.append(f"index {i} out of range")
            return errs
    for i, g in zip(idx, got_score):
        if not np.isfinite(s[i]) or s[i] <= tau - tol:
            errs.append(f"index {i} score {s[i]} not above tau={tau}")
        if not (abs(np.exp(float(g)) - np.exp(s[i])) <= rt * np.exp(s[i])):
            errs.append(f"index {i}: score {g} vs oracle {s[i]}")
    for a in range(len(idx)):
        for b in range(a + 1, len(idx)):
            if s[idx[a]] < s[idx[b]] - tol:
                errs.append(f"order: {idx[a]} ({s[idx[a]]}) before {idx[b]} ({s[idx[b]]})")
            elif s[idx[a]] == s[idx[b]] and idx[a] > idx[b]:
                errs.append(f"tie order: {idx[a]} before {idx[b]}")
    chosen = set(idx)
    worst = min((s[i] for i in idx), default=np.inf)
    for i in range(first, len(s)):
        if i in chosen or not np.isfinite(s[i]) or s[i] <= tau + tol:
            continue
        if len(idx) < n:
            errs.append(f"missing candidate {i} ({s[i]}) with only {len(idx)} chosen")
        elif s[i] > worst + tol:
            errs.append(f"candidate {i} ({s[i]}) beats chosen worst {worst}")
    return errs
