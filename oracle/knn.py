"""FP64 oracle of the instance-based Tier 2 model: IBK, the k-nearest-neighbour
learner that the paper settles on (Section 3.4 describes it; Section 6 picks
it; its results use k = 10).  Test infrastructure only (see the package
docstring).

Per optimisation o the model is a database of every before/after pair of o in
the training kernels (Sections 2 and 3.3): the before version's feature vector
and the measured log-speedup of adding o.  A prediction for a feature vector
is formed from the k stored vectors nearest to it in Euclidean distance
(Section 3.4).

Readings of the paper taken here:
  * the feature vectors are the standardised Tier 1 features z, as for the
    linear model (Section 3.4 does not say how IBK scales attributes);
  * the paper predicts with the mode of the neighbours' labels; a real-valued
    label has no useful mode, so the prediction is the mean of the k labels;
  * equal distances: the sample stored first is nearer (an optimisation's
    samples are stored kernel by kernel, then by before-version S);
  * fewer than k samples: all of them.
"""
from __future__ import annotations

import numpy as np

from .plain import candidate_pairs, column_stats, compose, features, pair_labels, standardize, suggest, TAU, N_SUGGEST

K_NEIGHBOURS = 10


def database(train, D: int) -> dict:
    """The training step of IBK (Section 3.4: every labelled instance is
    recorded), per global optimisation id, with the training features'
    column statistics."""
    x = features(train.counters, train.cycles)
    mu, sigma = column_stats(x)
    z = standardize(x, mu, sigma)
    opt, before, after, *_ = candidate_pairs(train.nopts, train.opt_ids, train.opt_off, train.row_off)
    y = pair_labels(train.cycles, before, after)
    db = {"mu": mu, "sigma": sigma, "D": D, "Z": {}, "y": {}}
    for o in range(D):
        sel = np.flatnonzero(opt == o)
        if sel.size:
            db["Z"][o] = z[before[sel]]
            db["y"][o] = y[sel]
    return db


def neighbours(Z: np.ndarray, q: np.ndarray, k: int = K_NEIGHBOURS):
    """Indices of the k rows of Z nearest to q (Euclidean), nearest first,
    earlier rows first among equal distances; and their squared distances."""
    d2 = ((Z - q[None, :]) ** 2).sum(axis=1)
    order = np.lexsort((np.arange(len(d2)), d2))[:k]
    return order, d2[order]


def predict_one(db: dict, z: np.ndarray, o: int, k: int = K_NEIGHBOURS) -> float:
    """Predicted log-speedup of adding global optimisation o to a version with
    standardised features z: the mean label of its k nearest samples."""
    if o not in db["Z"]:
        raise KeyError(f"optimisation {o} has no training samples")
    idx, _ = neighbours(db["Z"][o], z, k)
    return float(np.mean(db["y"][o][idx]))


def predict_grid(db: dict, batch, k: int = K_NEIGHBOURS, Bmax: int | None = None) -> np.ndarray:
    """Every single-optimisation prediction of a batch, laid out as the
    linear model's grid: grid[row(k,S), b] for b < B_k not in S, NaN
    elsewhere."""
    z = standardize(features(batch.counters, batch.cycles), db["mu"], db["sigma"])
    Bmax = int(max(batch.nopts, default=0)) if Bmax is None else Bmax
    grid = np.full((len(z), Bmax), np.nan)
    for kk in range(len(batch.nopts)):
        B = int(batch.nopts[kk])
        r0 = int(batch.row_off[kk])
        ids = batch.opt_ids[int(batch.opt_off[kk]):int(batch.opt_off[kk + 1])]
        for S in range(1 << B):
            for b in range(B):
                if not (S >> b) & 1:
                    grid[r0 + S, b] = predict_one(db, z[r0 + S], int(ids[b]), k)
    return grid


def run(db: dict, batch, k: int = K_NEIGHBOURS, tau: float = TAU, n: int = N_SUGGEST):
    """The scoring path with IBK as Tier 2: grid, composed table, suggestions."""
    grid = predict_grid(db, batch, k)
    table = compose(grid, batch)
    return grid, table, suggest(table, batch, tau, n)
