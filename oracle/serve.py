"""FP64 oracle of the serving rule that puts a learned surrogate in front of
the plain method.  Test infrastructure only (see the package docstring).

The paper has no surrogate: its Tier 2 models (Section 2) stay the reference,
and a surrogate's answer for a kernel is kept only where the plain models
confirm it.  The rule (a reading: the paper is silent), per kernel with
surrogate table Ls[S] and plain composed table L[S], S in [0, 2^B):

  1. the surrogate's list: Tier 3's ranking (Section 2) of Ls over S >= 1,
     strictly above tau, top n;
  2. the threshold band: when that list holds fewer than n subsets, every
     other S >= 1 with Ls[S] >= tau - band (those the threshold alone left
     out); none when the list is full;
  3. more than ``cap`` band subsets: the kernel falls back;
  4. otherwise the kernel falls back when some listed or band subset has
     |Ls[S] - L[S]| > tol (or a non-finite difference);
  5. it also falls back unless the plain values keep Tier 3's threshold
     (Section 2: only choices above it): every listed subset has L[S] > tau
     and no band subset has L[S] > tau;
  6. a kernel that falls back gets the plain answer (Tier 3 on L); the others
     keep the surrogate's subsets with their plain values L[S], sorted by
     them (Tier 3's order: descending, equal values by smaller S).  A kept
     answer is then exactly Tier 3's ranking of the plain values over the
     judged subsets.
"""
from __future__ import annotations

import numpy as np

from .plain import N_SUGGEST, TAU, rank

TOL = 0.1
BAND = 0.1
CAP = 16


def band(sur, listed, tau: float = TAU, n: int = N_SUGGEST, band_width: float = BAND):
    """Step 2: ascending subsets S >= 1 outside the surrogate's list with
    Ls[S] >= tau - band_width, for a list shorter than n; else empty."""
    if len(listed) >= n:
        return []
    s = np.asarray(sur, dtype=np.float64)
    keep = set(listed)
    return [S for S in range(1, len(s)) if S not in keep and s[S] >= tau - band_width]


def serve_kernel(sur, plain, tau: float = TAU, n: int = N_SUGGEST, tol: float = TOL,
                 band_width: float = BAND, cap: int = CAP):
    """Steps 1-5 for one kernel.  Returns (fallback, answer, judged) with
    answer a list of (S, plain value) and judged the subsets checked."""
    sur = np.asarray(sur, dtype=np.float64)
    plain = np.asarray(plain, dtype=np.float64)
    listed = [S for S, _ in rank(sur, tau, n, first=1)]
    extra = band(sur, listed, tau, n, band_width)
    judged = listed + extra
    if len(extra) > cap:
        return True, rank(plain, tau, n, first=1), judged
    if any(not abs(sur[S] - plain[S]) <= tol for S in judged):
        return True, rank(plain, tau, n, first=1), judged
    if any(not plain[S] > tau for S in listed) or any(plain[S] > tau for S in extra):
        return True, rank(plain, tau, n, first=1), judged
    kept = sorted(listed, key=lambda S: (-plain[S], S))
    return False, [(S, float(plain[S])) for S in kept], judged


def serve(sur_tables, plain_tables, **kw):
    """serve_kernel over kernels (sequences of per-kernel tables)."""
    return [serve_kernel(s, p, **kw) for s, p in zip(sur_tables, plain_tables)]
