"""FP64 oracle of the model-tree Tier 2 learner, M5P (Section 3.4), used per
optimisation in place of the linear model.  Test infrastructure only (see the
package docstring).

Section 3.4 gives the method's outline, after Quinlan's M5: grow an ordinary
regression tree; fit a multivariate linear model at every node from the
node's training cases, restricted to the features that the subtree below the
node tests; the leaves take these models; then prune and smooth.  The details
it leaves open are taken from the M5 method itself (Quinlan 1992, the paper's
reference for M5):

  growth     binary splits z_j <= t of one feature; t is the midpoint of two
             adjacent distinct training values of z_j.  The split chosen
             maximises the standard-deviation reduction
                 SDR = sd(T) - |T_l|/|T| sd(T_l) - |T_r|/|T| sd(T_r)
             (population standard deviations of the labels).  A node is not
             split when it holds fewer than 2 * MIN_LEAF cases, when its
             labels' sd is at most SD_FRAC of the root's, or when no split leaves
             MIN_LEAF cases on each side.
  error      a model's estimated error is its mean absolute residual on the
             node's training cases times (n + v) / (n - v), n cases, v
             parameters (features + intercept); infinite when n <= v.
  pruning    bottom-up: an interior node becomes a leaf carrying its own
             model when that model's estimated error is no larger than the
             case-weighted mean of its (already pruned) children's.
  smoothing  a prediction starts as the leaf model's value and, at every
             ancestor on the way back to the root, becomes
                 (n_c * p + K * q) / (n_c + K),
             q the ancestor's model at the query, n_c the training cases of
             the child the query came from, K = SMOOTH_K.

Readings of the paper taken here:
  * inputs: the standardised Tier 1 features and the before/after log-speedup
    labels of the linear model (Sections 2, 3.3);
  * node models are ordinary least squares with an intercept (no penalty), and
    M5's greedy deletion of model terms is not applied; a feature of A whose
    node-centred column lies in the span of the features kept before it (its
    residual sum of squares after regressing on them is at most DROP times its
    own) is left out, so the solution is unique even when counters are
    collinear, and the error estimate counts the kept parameters only;
  * MIN_LEAF = 4 cases, SD_FRAC = 0.05, K = 15;
  * ties: split candidates whose SDR is within TIE * sd(root) of the best are
    equal and the first in (feature, threshold) order wins; a pruning
    comparison within TIE * sd(root) prunes.  (Exact ties are common: two
    features that order a node's cases alike give the same SDR, up to the
    rounding of the sums.)

A tree is stored in preorder (node, its left subtree, its right subtree):
feat (-1 at a leaf), thr, left, right (-1 at a leaf), n (training cases),
and per node the model (feature list A, coefficients, intercept).
"""
from __future__ import annotations

import numpy as np

from .plain import candidate_pairs, column_stats, compose, features, pair_labels, standardize, suggest, TAU, N_SUGGEST

MIN_LEAF = 4
SD_FRAC = 0.05
SMOOTH_K = 15.0
TIE = 1e-9
DROP = 1e-9


def label_sd(y: np.ndarray) -> float:
    """Population standard deviation."""
    return float(np.sqrt(np.mean((y - y.mean()) ** 2))) if len(y) else 0.0


def best_split(Z: np.ndarray, y: np.ndarray, min_leaf: int, tol: float):
    """The M5 split of the cases (Z, y): (feature, threshold, SDR) or None.

    For every feature the cases are sorted by value; a split after the i-th
    sorted case (i = min_leaf .. n - min_leaf) is admissible when the i-th and
    (i+1)-th values differ.  Side standard deviations come from running sums
    of the node-centred labels and their squares."""
    n, E = Z.shape
    if n < 2 * min_leaf:
        return None
    yc = y - y.mean()
    sd_t = float(np.sqrt(np.mean(yc * yc)))
    order = np.argsort(Z, axis=0, kind="stable")
    v = np.take_along_axis(Z, order, axis=0)
    Y = yc[order]
    s1 = np.cumsum(Y, axis=0)
    s2 = np.cumsum(Y * Y, axis=0)
    i = np.arange(min_leaf, n - min_leaf + 1)          # cases on the left
    nl = i[:, None].astype(np.float64)
    nr = n - nl
    l1, l2 = s1[i - 1], s2[i - 1]
    r1, r2 = s1[-1] - l1, s2[-1] - l2
    sdl = np.sqrt(np.maximum(l2 / nl - (l1 / nl) ** 2, 0.0))
    sdr_ = np.sqrt(np.maximum(r2 / nr - (r1 / nr) ** 2, 0.0))
    sdr = sd_t - (nl / n) * sdl - (nr / n) * sdr_
    ok = v[i - 1] < v[i]
    sdr = np.where(ok, sdr, -np.inf)
    best = sdr.max() if sdr.size else -np.inf
    if not np.isfinite(best):
        return None
    # first (feature, position) within tol of the best
    hit = (sdr >= best - tol).T.ravel()
    flat = int(np.argmax(hit))
    j, p = divmod(flat, len(i))
    thr = 0.5 * (v[i[p] - 1, j] + v[i[p], j])
    return j, float(thr), float(sdr[p, j])


def grow(Z: np.ndarray, y: np.ndarray, min_leaf: int = MIN_LEAF, sd_frac: float = SD_FRAC):
    """The unpruned regression tree, preorder: list of dicts with the cases
    (indices into Z), feat, thr, left, right."""
    sd_root = label_sd(y)
    tol = TIE * sd_root
    nodes = []
    stack = [(np.arange(len(y)), -1, 0)]          # (cases, parent, side)
    while stack:
        idx, parent, side = stack.pop()
        me = len(nodes)
        nodes.append({"idx": idx, "n": len(idx), "feat": -1, "thr": np.nan, "left": -1, "right": -1})
        if parent >= 0:
            nodes[parent]["left" if side == 0 else "right"] = me
        if len(idx) < 2 * min_leaf or label_sd(y[idx]) <= sd_frac * sd_root:
            continue
        s = best_split(Z[idx], y[idx], min_leaf, tol)
        if s is None:
            continue
        j, thr, _ = s
        nodes[me]["feat"], nodes[me]["thr"] = j, thr
        go_left = Z[idx, j] <= thr
        stack.append((idx[~go_left], me, 1))
        stack.append((idx[go_left], me, 0))       # popped first: preorder
    return nodes


def subtree_features(nodes):
    """A(node): the sorted features tested at the interior nodes of each
    node's subtree (empty at a leaf)."""
    A = [set() for _ in nodes]
    for i in reversed(range(len(nodes))):         # children follow parents
        nd = nodes[i]
        if nd["feat"] >= 0:
            A[i] = {nd["feat"]} | A[nd["left"]] | A[nd["right"]]
    return [sorted(a) for a in A]


def independent_features(Z: np.ndarray, A):
    """The features of A, in order, whose node-centred column is not (up to
    DROP) in the span of the features kept before it."""
    Xc = Z[:, A] - Z[:, A].mean(axis=0)
    keep, basis = [], np.zeros((len(Xc), 0))    # orthonormal basis of the kept columns
    for q in range(len(A)):
        x = Xc[:, q]
        ss = float(x @ x)
        res = x.copy()
        for _ in range(2):                        # projected out twice, for accuracy
            res -= basis @ (basis.T @ res)
        rss = float(res @ res)
        if ss > 0 and rss > DROP * ss:
            keep.append(q)
            basis = np.hstack([basis, (res / np.sqrt(rss))[:, None]])
    return [A[q] for q in keep]


def fit_node_model(Z: np.ndarray, y: np.ndarray, A):
    """Least-squares model with an intercept on the independent features of A
    (see independent_features; coefficient 0 for the others), and its M5
    error estimate."""
    n = len(y)
    K = independent_features(Z, A) if A else []
    X = np.hstack([Z[:, K], np.ones((n, 1))])
    coef = np.linalg.lstsq(X, y, rcond=None)[0]
    w = np.zeros(len(A))
    for j, f in enumerate(K):
        w[A.index(f)] = coef[j]
    mae = float(np.mean(np.abs(y - X @ coef)))
    v = len(K) + 1
    est = (n + v) / (n - v) * mae if n > v else np.inf
    return {"A": list(A), "w": w, "b": float(coef[-1]), "est": est}


def build(Z: np.ndarray, y: np.ndarray, min_leaf: int = MIN_LEAF, sd_frac: float = SD_FRAC):
    """Section 3.4's M5P steps: grow, node models on the subtree's features,
    prune.  Returns the pruned tree in preorder (see the module docstring)."""
    nodes = grow(Z, y, min_leaf, sd_frac)
    A = subtree_features(nodes)
    models = [fit_node_model(Z[nd["idx"]], y[nd["idx"]], A[i]) for i, nd in enumerate(nodes)]
    tol = TIE * label_sd(y)
    leaf = [nd["feat"] < 0 for nd in nodes]
    est = [0.0] * len(nodes)
    for i in reversed(range(len(nodes))):
        nd = nodes[i]
        if leaf[i]:
            est[i] = models[i]["est"]
            continue
        L, R = nd["left"], nd["right"]
        sub = (nodes[L]["n"] * est[L] + nodes[R]["n"] * est[R]) / nd["n"]
        if models[i]["est"] <= sub + tol:
            leaf[i] = True
            est[i] = models[i]["est"]
        else:
            est[i] = sub
    # the pruned tree, renumbered in preorder
    out = {"feat": [], "thr": [], "left": [], "right": [], "n": [], "model": []}
    stack = [(0, -1, 0)]
    while stack:
        i, parent, side = stack.pop()
        me = len(out["feat"])
        nd = nodes[i]
        out["feat"].append(-1 if leaf[i] else nd["feat"])
        out["thr"].append(np.nan if leaf[i] else nd["thr"])
        out["left"].append(-1)
        out["right"].append(-1)
        out["n"].append(nd["n"])
        out["model"].append(models[i])
        if parent >= 0:
            out["left" if side == 0 else "right"][parent] = me
        if not leaf[i]:
            stack.append((nd["right"], me, 1))
            stack.append((nd["left"], me, 0))
    for key in ("feat", "left", "right", "n"):
        out[key] = np.asarray(out[key], dtype=np.int64)
    out["thr"] = np.asarray(out["thr"], dtype=np.float64)
    return out


def model_value(m: dict, z: np.ndarray) -> float:
    return float(z[m["A"]] @ m["w"] + m["b"]) if m["A"] else m["b"]


def predict_one(tree: dict, z: np.ndarray, smooth_k: float = SMOOTH_K):
    """Smoothed prediction for the standardised vector z, and the smallest
    |z_f - t| over the tests on its path (how far z is from switching)."""
    path, i, margin = [0], 0, np.inf
    while tree["feat"][i] >= 0:
        f, t = tree["feat"][i], tree["thr"][i]
        margin = min(margin, abs(z[f] - t))
        i = tree["left"][i] if z[f] <= t else tree["right"][i]
        path.append(i)
    p = model_value(tree["model"][path[-1]], z)
    for a, c in zip(reversed(path[:-1]), reversed(path[1:])):
        nc = tree["n"][c]
        p = (nc * p + smooth_k * model_value(tree["model"][a], z)) / (nc + smooth_k)
    return p, margin


def fit(train, D: int, min_leaf: int = MIN_LEAF, smooth_k: float = SMOOTH_K) -> dict:
    """Tier 2 training with M5P: one tree per global optimisation from its
    before/after pairs (same features and labels as the linear model)."""
    x = features(train.counters, train.cycles)
    mu, sigma = column_stats(x)
    z = standardize(x, mu, sigma)
    opt, before, after, *_ = candidate_pairs(train.nopts, train.opt_ids, train.opt_off, train.row_off)
    y = pair_labels(train.cycles, before, after)
    trees = {}
    for o in range(D):
        sel = np.flatnonzero(opt == o)
        if sel.size:
            trees[o] = build(z[before[sel]], y[sel], min_leaf)
    return {"mu": mu, "sigma": sigma, "D": D, "trees": trees, "smooth_k": smooth_k}


def predict_grid(model: dict, batch, Bmax: int | None = None):
    """Every single-optimisation prediction of a batch in the linear model's
    grid layout (NaN where b is in S or b >= B_k), and the margin of each."""
    z = standardize(features(batch.counters, batch.cycles), model["mu"], model["sigma"])
    Bmax = int(max(batch.nopts, default=0)) if Bmax is None else Bmax
    grid = np.full((len(z), Bmax), np.nan)
    margin = np.full((len(z), Bmax), np.inf)
    for kk in range(len(batch.nopts)):
        B, r0 = int(batch.nopts[kk]), int(batch.row_off[kk])
        ids = batch.opt_ids[int(batch.opt_off[kk]):int(batch.opt_off[kk + 1])]
        for S in range(1 << B):
            for b in range(B):
                if not (S >> b) & 1:
                    tree = model["trees"][int(ids[b])]
                    grid[r0 + S, b], margin[r0 + S, b] = predict_one(tree, z[r0 + S], model["smooth_k"])
    return grid, margin


def run(model: dict, batch, tau: float = TAU, n: int = N_SUGGEST):
    """The scoring path with M5P as Tier 2: grid, composed table, suggestions."""
    grid, _ = predict_grid(model, batch)
    table = compose(grid, batch)
    return grid, table, suggest(table, batch, tau, n)
