"""FP64 oracle of the plain suggestion method (Tiers 1-3 of Section 2).

Test infrastructure only (see the package docstring).

Notation
  K kernels; kernel k has B_k binary optimisations with global ids O_k[0..B_k),
  ascending, and one profiled row per version S in [0, 2^B_k) (the subset
  bitmask over its local bits), stored at row row_off[k] + S (Section 3.3:
  every combination of the optimisations is a version).
  E counter events per row plus a separate cycle count.

Readings of the paper taken here (the paper is silent or loose on these):
  * features are the natural log of counter / cycles (Section 2 normalises by
    the cycle count; the log makes the multiplicative counters additive),
    then standardised per column with the training rows' mean and population
    standard deviation (a column with sigma < 1e-12 gets sigma = 1);
  * the quantity learned per optimisation is the log-speedup of adding it,
    ln cyc(before) - ln cyc(after), from every before/after pair in the
    training kernels (Sections 2 and 3.3: 2^(B-1) pairs per optimisation);
  * the regression family is linear (Section 3.4) with a ridge penalty on the
    feature weights only, sum-of-squares loss, intercept unpenalised;
  * the speedup of a subset S is composed along the ascending chain of its
    bits from the baseline version;
  * ranking keeps entries strictly above the threshold tau (log of 1.05),
    sorted by predicted benefit, ties broken by the smaller index, first n
    (Section 2, Tier 3).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

TAU = float(np.log(1.05))
LAMBDA = 1e-2
N_SUGGEST = 3
SIGMA_FLOOR = 1e-12


# ---------------------------------------------------------------- Tier 1 ----
def features(counters, cycles) -> np.ndarray:
    """Section 2, Tier 1: divide every counter by the run's cycle count so the
    features do not depend on the run time; x[r, j] = ln(c[r, j] / cyc[r])."""
    c = np.asarray(counters, dtype=np.float64)
    cyc = np.asarray(cycles, dtype=np.float64)
    return np.log(c / cyc[:, None])


def column_stats(x: np.ndarray):
    """Column mean and population standard deviation over the training rows."""
    mu = x.mean(axis=0)
    sigma = np.sqrt(((x - mu) ** 2).mean(axis=0))
    sigma = np.where(sigma < SIGMA_FLOOR, 1.0, sigma)
    return mu, sigma


def standardize(x: np.ndarray, mu: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    return (x - mu) / sigma


# ------------------------------------------------------- training pairs ----
def candidate_pairs(nopts, opt_ids, opt_off, row_off):
    """Before/after pairs (Section 2, optimisation database; Section 3.3).

    For every kernel k, version S and local bit b not in S there is one pair:
    before = version S, after = version S with b added; it teaches global
    optimisation O_k[b].  Returns arrays (opt, before_row, after_row, kernel,
    S, b), ordered by kernel, then b, then S.
    """
    opt, before, after, kern, subs, bit = [], [], [], [], [], []
    for k in range(len(nopts)):
        B = int(nopts[k])
        O = np.asarray(opt_ids[opt_off[k]:opt_off[k + 1]])
        S = np.arange(1 << B, dtype=np.int64)
        for b in range(B):
            without = S[(S >> b) & 1 == 0]
            opt.append(np.full(len(without), O[b], dtype=np.int64))
            before.append(row_off[k] + without)
            after.append(row_off[k] + (without | (1 << b)))
            kern.append(np.full(len(without), k, dtype=np.int64))
            subs.append(without)
            bit.append(np.full(len(without), b, dtype=np.int64))
    if not opt:
        e = np.zeros(0, dtype=np.int64)
        return e, e, e, e, e, e
    return tuple(np.concatenate(a) for a in (opt, before, after, kern, subs, bit))


def pair_labels(cycles, before, after) -> np.ndarray:
    """Measured log-speedup of a pair: ln cyc(before) - ln cyc(after)."""
    cyc = np.asarray(cycles, dtype=np.float64)
    return np.log(cyc[before]) - np.log(cyc[after])


# --------------------------------------------------------------- Tier 2 ----
def ridge_fit(Z: np.ndarray, y: np.ndarray, lam: float) -> np.ndarray:
    """Linear regression with a ridge penalty (Section 3.4's regression family).

    Minimises sum (y - [Z, 1] w)^2 + lam * sum_{j < E} w_j^2 by solving the
    normal equations ([Z,1]^T [Z,1] + lam diag(1,..,1,0)) w = [Z,1]^T y with a
    Cholesky factorisation.  Returns w of length E + 1 (intercept last).
    """
    n, E = Z.shape
    X = np.hstack([Z, np.ones((n, 1))])
    A = X.T @ X
    A[np.arange(E), np.arange(E)] += lam
    r = X.T @ y
    L = np.linalg.cholesky(A)
    t = solve_triangular(L, r, lower=True)
    return solve_triangular(L.T, t, lower=False)


def fit(train, D: int, lam: float = LAMBDA) -> dict:
    """Tier 2 training (Section 2): standardise the training features, then one
    ridge model per optimisation from all of its before/after pairs (Section 7:
    a model for each optimisation in the database).  Optimisations without a
    pair stay untrained (count 0, weights NaN)."""
    x = features(train.counters, train.cycles)
    mu, sigma = column_stats(x)
    z = standardize(x, mu, sigma)
    opt, before, after, *_ = candidate_pairs(train.nopts, train.opt_ids,
                                             train.opt_off, train.row_off)
    y = pair_labels(train.cycles, before, after)
    E = z.shape[1]
    W = np.full((D, E + 1), np.nan)
    counts = np.zeros(D, dtype=np.int64)
    for o in range(D):
        sel = opt == o
        counts[o] = int(sel.sum())
        if counts[o]:
            W[o] = ridge_fit(z[before[sel]], y[sel], lam)
    return {"mu": mu, "sigma": sigma, "W": W, "counts": counts, "lam": lam}


def predict_grid(model: dict, batch, Bmax: int | None = None) -> np.ndarray:
    """Predicted log-speedup of adding each optimisation to each version
    (Section 5's evaluation: every version without an optimisation is scored
    for it).  grid[r, b] = w_{O_k[b]} . [z_r, 1] for b not in S, NaN for b in S."""
    z = standardize(features(batch.counters, batch.cycles), model["mu"], model["sigma"])
    K = len(batch.nopts)
    if Bmax is None:
        Bmax = int(max(batch.nopts)) if K else 0
    grid = np.full((z.shape[0], Bmax), np.nan)
    W = model["W"]
    for k in range(K):
        B = int(batch.nopts[k])
        O = batch.opt_ids[batch.opt_off[k]:batch.opt_off[k + 1]]
        r0 = int(batch.row_off[k])
        S = np.arange(1 << B)
        for b in range(B):
            without = S[(S >> b) & 1 == 0]
            w = W[O[b]]
            grid[r0 + without, b] = z[r0 + without] @ w[:-1] + w[-1]
    return grid


def compose(grid: np.ndarray, batch) -> np.ndarray:
    """Predicted log-speedup of applying subset S to the baseline version:
    L[S] = sum over the bits b of S in ascending order of grid[S & (2^b - 1), b],
    i.e. add the optimisations one at a time along the ascending chain
    (the paper predicts single optimisations only; this chain is the reading
    used for subsets).  L[0] = 0."""
    L = np.zeros(grid.shape[0])
    for k in range(len(batch.nopts)):
        B = int(batch.nopts[k])
        r0 = int(batch.row_off[k])
        S = np.arange(1 << B)
        acc = np.zeros(1 << B)
        for b in range(B):
            has = S[(S >> b) & 1 == 1]
            acc[has] += grid[r0 + (has & ((1 << b) - 1)), b]
        L[r0:r0 + (1 << B)] = acc
    return L


# --------------------------------------------------------------- Tier 3 ----
def rank(scores, tau: float = TAU, n: int = N_SUGGEST, first: int = 0):
    """Tier 3 (Section 2): keep the entries whose predicted benefit is above
    the threshold, sort by expected benefit (ties: smaller index first) and
    return the first n as (index, score) pairs.  Indices below ``first`` are
    not candidates."""
    s = np.asarray(scores, dtype=np.float64)
    cand = [i for i in range(first, len(s)) if s[i] > tau]
    cand = sorted(cand, key=lambda i: (-s[i], i))
    return [(i, float(s[i])) for i in cand[:n]]


def suggest(table: np.ndarray, batch, tau: float = TAU, n: int = N_SUGGEST):
    """Per kernel: the top-n subsets S != 0 of its composed table above tau."""
    out = []
    for k in range(len(batch.nopts)):
        r0, r1 = int(batch.row_off[k]), int(batch.row_off[k + 1])
        out.append(rank(table[r0:r1], tau, n, first=1))
    return out


def suggest_rows(grid: np.ndarray, tau: float = TAU, n: int = N_SUGGEST):
    """Per version (row): the top-n single optimisations (local bits) above tau,
    the tool's output for one profiled kernel in the paper's own form."""
    return [rank(grid[r], tau, n) for r in range(grid.shape[0])]


def run(model: dict, batch, tau: float = TAU, n: int = N_SUGGEST):
    """The whole scoring path: grid, composed table and suggestions."""
    grid = predict_grid(model, batch)
    table = compose(grid, batch)
    return grid, table, suggest(table, batch, tau, n)


# -------------------------------------------------------------- metrics ----
def mape(table: np.ndarray, truth: np.ndarray, batch) -> float:
    """Mean absolute percentage error of the predicted speedups e^L against the
    true speedups e^T over every (kernel, S != 0)."""
    m = np.ones(len(table), dtype=bool)
    m[np.asarray(batch.row_off[:-1], dtype=np.int64)] = False
    a, t = np.exp(table[m]), np.exp(truth[m])
    return float(np.mean(np.abs(a - t) / t)) if m.any() else 0.0


def step_truth(truth: np.ndarray, batch, Bmax: int | None = None) -> np.ndarray:
    """True log-speedup of adding local bit b to version S: T[S|b] - T[S]."""
    K = len(batch.nopts)
    if Bmax is None:
        Bmax = int(max(batch.nopts)) if K else 0
    out = np.full((len(truth), Bmax), np.nan)
    for k in range(K):
        B = int(batch.nopts[k])
        r0 = int(batch.row_off[k])
        S = np.arange(1 << B)
        for b in range(B):
            without = S[(S >> b) & 1 == 0]
            out[r0 + without, b] = truth[r0 + (without | (1 << b))] - truth[r0 + without]
    return out


def sign_accuracy(pred: np.ndarray, true: np.ndarray) -> float:
    """Table 3's measure: share of predictions on the same side of a speedup of
    1 (log-speedup 0) as the actual value."""
    m = np.isfinite(pred) & np.isfinite(true)
    return float(np.mean((pred[m] > 0) == (true[m] > 0))) if m.any() else 0.0


def acex(pred: np.ndarray, true: np.ndarray, qs=(0.05, 0.5, 0.95)):
    """Quantiles of actual / expected speedup, Section 5's AC/EX ratio."""
    m = np.isfinite(pred) & np.isfinite(true)
    r = np.exp(true[m]) / np.exp(pred[m])
    return [float(np.quantile(r, q)) for q in qs] if m.any() else [np.nan] * len(qs)


# -------------------------------------------------------------- batches ----
class SubBatch:
    """Kernels ``ks`` of a batch, re-laid out contiguously."""

    def __init__(self, batch, ks):
        ks = list(ks)
        self.nopts = np.asarray([batch.nopts[k] for k in ks], dtype=np.int64)
        self.opt_ids = (np.concatenate([batch.opt_ids[batch.opt_off[k]:batch.opt_off[k + 1]]
                                        for k in ks]) if ks else np.zeros(0, np.int64))
        self.opt_off = np.concatenate([[0], np.cumsum(self.nopts)]).astype(np.int64)
        self.row_off = np.concatenate([[0], np.cumsum(1 << self.nopts)]).astype(np.int64)
        rows = (np.concatenate([np.arange(batch.row_off[k], batch.row_off[k + 1]) for k in ks])
                if ks else np.zeros(0, np.int64))
        self.counters = batch.counters[rows]
        self.cycles = batch.cycles[rows]
        self.truth = batch.truth[rows] if getattr(batch, "truth", None) is not None else None


def leave_one_kernel_out(batch, D: int, lam: float = LAMBDA, tau: float = TAU,
                         n: int = N_SUGGEST):
    """Cross-program protocol (Section 5, experiments 5 and 6: train on one
    program, test on another): for each kernel k, fit on every other kernel,
    then score and rank kernel k.  Returns one dict per fold."""
    folds = []
    K = len(batch.nopts)
    for k in range(K):
        train = SubBatch(batch, [i for i in range(K) if i != k])
        test = SubBatch(batch, [k])
        model = fit(train, D, lam)
        grid, table, sugg = run(model, test, tau, n)
        folds.append({"model": model, "grid": grid, "table": table,
                      "suggestions": sugg, "test": test})
    return folds
