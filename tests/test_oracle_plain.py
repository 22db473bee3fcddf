"""Pins of the FP64 oracle of the plain method against closed forms,
independent numerical routes, brute force on tiny inputs and invariants.
CPU only."""
import itertools
import math

import numpy as np
import pytest
from scipy.linalg import hadamard

from oracle import plain as P
from oracle.checks import check_list


def small_batch(nopts, E=5, seed=0):
    """A hand-laid ragged batch with random positive counters."""
    rng = np.random.default_rng(seed)
    nopts = np.asarray(nopts, dtype=np.int64)
    D = 8
    opt_ids = np.concatenate([np.sort(rng.choice(D, size=b, replace=False)) for b in nopts]) \
        if len(nopts) else np.zeros(0, np.int64)
    opt_off = np.concatenate([[0], np.cumsum(nopts)]).astype(np.int64)
    row_off = np.concatenate([[0], np.cumsum(1 << nopts)]).astype(np.int64)
    N = int(row_off[-1])

    class B:
        pass
    b = B()
    b.nopts, b.opt_ids, b.opt_off, b.row_off = nopts, opt_ids.astype(np.int64), opt_off, row_off
    b.counters = np.exp(rng.normal(5, 1, size=(N, E)))
    b.cycles = np.exp(rng.normal(8, 1, size=N))
    b.truth = rng.normal(0, 0.1, size=N)
    return b, D


# --------------------------------------------------------------- Tier 1 ----
def test_features_closed_form():
    c = np.array([[math.e ** 3, math.e, 5.0]])
    cyc = np.array([math.e ** 2])
    x = P.features(c, cyc)
    np.testing.assert_allclose(x[0], [1.0, -1.0, math.log(5.0) - 2.0], rtol=0, atol=1e-15)


def test_features_row_scale_invariance():
    b, _ = small_batch([3, 2], E=7)
    x = P.features(b.counters, b.cycles)
    alpha = np.exp(np.random.default_rng(1).normal(0, 2, size=len(b.cycles)))
    x2 = P.features(b.counters * alpha[:, None], b.cycles * alpha)
    np.testing.assert_allclose(x2, x, rtol=0, atol=4 * np.finfo(float).eps * np.abs(x).max())


def test_column_stats_known_values_and_standardisation():
    x = np.array([[1.0, 7.0], [2.0, 7.0], [3.0, 7.0], [4.0, 7.0]])
    mu, sigma = P.column_stats(x)
    np.testing.assert_allclose(mu, [2.5, 7.0])
    # population (ddof 0) standard deviation; a constant column gets sigma 1
    np.testing.assert_allclose(sigma, [math.sqrt(1.25), 1.0])
    z = P.standardize(x, mu, sigma)
    np.testing.assert_array_equal(z[:, 1], 0.0)
    rng = np.random.default_rng(3)
    x = rng.normal(rng.uniform(-5, 5, 9), rng.uniform(0.1, 3, 9), size=(500, 9))
    z = P.standardize(x, *P.column_stats(x))
    assert np.abs(z.mean(0)).max() < 1e-12
    assert np.abs(z.var(0) - 1).max() < 1e-12


# ------------------------------------------------------- training pairs ----
@pytest.mark.parametrize("nopts", [[0], [1], [3], [2, 0, 3, 1], [4, 4]])
def test_candidate_pairs_bruteforce(nopts):
    b, _ = small_batch(nopts)
    opt, before, after, kern, S, bit = P.candidate_pairs(b.nopts, b.opt_ids, b.opt_off, b.row_off)
    assert len(opt) == sum(n * (1 << n) // 2 for n in nopts)
    got = set(zip(opt.tolist(), before.tolist(), after.tolist()))
    want = set()
    for k, B in enumerate(nopts):
        O = b.opt_ids[b.opt_off[k]:b.opt_off[k + 1]]
        versions = [frozenset(c) for r in range(B + 1) for c in itertools.combinations(range(B), r)]
        for s in versions:
            for t in versions:
                if s < t and len(t - s) == 1:
                    (added,) = tuple(t - s)
                    rs = b.row_off[k] + sum(1 << i for i in s)
                    rt = b.row_off[k] + sum(1 << i for i in t)
                    want.add((int(O[added]), int(rs), int(rt)))
    assert got == want


def test_pair_labels_telescope():
    b, _ = small_batch([4])
    opt, before, after, kern, S, bit = P.candidate_pairs(b.nopts, b.opt_ids, b.opt_off, b.row_off)
    y = P.pair_labels(b.cycles, before, after)
    lab = {(int(s), int(bb)): v for s, bb, v in zip(S, bit, y)}
    for target in range(16):
        for order in itertools.permutations([i for i in range(4) if target >> i & 1]):
            s, tot = 0, 0.0
            for bb in order:
                tot += lab[(s, bb)]
                s |= 1 << bb
            assert abs(tot - (math.log(b.cycles[0]) - math.log(b.cycles[target]))) < 1e-12


# ---------------------------------------------------------------- ridge ----
def test_ridge_matches_augmented_least_squares():
    rng = np.random.default_rng(7)
    n, E, lam = 60, 9, 0.37
    Z = rng.normal(size=(n, E))
    y = rng.normal(size=n)
    w = P.ridge_fit(Z, y, lam)
    # independent route: QR/SVD least squares on the penalty-augmented system
    X = np.hstack([Z, np.ones((n, 1))])
    pen = np.sqrt(lam) * np.eye(E + 1)[:E]
    Xa = np.vstack([X, pen])
    ya = np.concatenate([y, np.zeros(E)])
    w2 = np.linalg.lstsq(Xa, ya, rcond=None)[0]
    np.testing.assert_allclose(w, w2, rtol=1e-10, atol=1e-12)
    # normal-equation residual
    A = X.T @ X + lam * np.diag(np.r_[np.ones(E), 0.0])
    res = A @ w - X.T @ y
    assert np.abs(res).max() <= 1e-10 * np.abs(X.T @ y).max()


def test_ridge_underdetermined_matches_augmented_least_squares():
    # fewer samples than features (the 2-kernel cross-program case)
    rng = np.random.default_rng(8)
    n, E, lam = 32, 40, 1e-2
    Z = rng.normal(size=(n, E))
    y = rng.normal(size=n)
    w = P.ridge_fit(Z, y, lam)
    X = np.hstack([Z, np.ones((n, 1))])
    Xa = np.vstack([X, np.sqrt(lam) * np.eye(E + 1)[:E]])
    w2 = np.linalg.lstsq(Xa, np.concatenate([y, np.zeros(E)]), rcond=None)[0]
    np.testing.assert_allclose(w, w2, rtol=1e-8, atol=1e-9)


def test_ridge_zero_penalty_is_ols():
    rng = np.random.default_rng(9)
    n, E = 80, 6
    Z = rng.normal(size=(n, E))
    y = Z @ rng.normal(size=E) + 0.3 + rng.normal(0, 0.1, n)
    w = P.ridge_fit(Z, y, 0.0)
    ols = np.linalg.lstsq(np.hstack([Z, np.ones((n, 1))]), y, rcond=None)[0]
    np.testing.assert_allclose(w, ols, rtol=1e-10, atol=1e-12)


def test_ridge_orthogonal_design_shrinkage():
    # Hadamard columns (minus the all-ones one) are centred and Z^T Z = n I,
    # so the ridge weights are beta * n / (n + lam) and the intercept is mean(y).
    n, E, lam = 16, 7, 2.5
    H = hadamard(n).astype(float)
    Z = H[:, 1:E + 1]
    beta = np.arange(1, E + 1) * 0.25 - 1.0
    c0 = 0.7
    y = Z @ beta + c0
    w = P.ridge_fit(Z, y, lam)
    np.testing.assert_allclose(w[:E], beta * n / (n + lam), rtol=1e-13, atol=1e-14)
    assert abs(w[E] - c0) < 1e-13


def test_ridge_intercept_not_penalised():
    rng = np.random.default_rng(10)
    Z = rng.normal(size=(30, 4))
    Z -= Z.mean(0)
    w = P.ridge_fit(Z, np.full(30, 3.25), 5.0)
    np.testing.assert_allclose(w, [0, 0, 0, 0, 3.25], atol=1e-12)


# ----------------------------------------------------- grid and compose ----
def test_predict_grid_masks_and_values():
    b, D = small_batch([3, 2], E=4)
    rng = np.random.default_rng(11)
    x = P.features(b.counters, b.cycles)
    model = {"mu": x.mean(0), "sigma": x.std(0), "W": rng.normal(size=(D, 5))}
    grid = P.predict_grid(model, b)
    z = (x - x.mean(0)) / x.std(0)
    for k in range(2):
        B = b.nopts[k]
        O = b.opt_ids[b.opt_off[k]:b.opt_off[k + 1]]
        for s in range(1 << B):
            r = b.row_off[k] + s
            for bb in range(3):
                if bb >= B or (s >> bb) & 1:
                    assert np.isnan(grid[r, bb])
                else:
                    want = sum(model["W"][O[bb], j] * z[r, j] for j in range(4)) + model["W"][O[bb], 4]
                    assert abs(grid[r, bb] - want) < 1e-12


def test_compose_telescopes_on_exact_steps():
    b, _ = small_batch([5, 1, 3, 0])
    T = np.random.default_rng(12).normal(size=int(b.row_off[-1]))
    grid = np.full((len(T), 5), np.nan)
    for k in range(4):
        B = b.nopts[k]
        r0 = b.row_off[k]
        for s in range(1 << B):
            for bb in range(B):
                if not (s >> bb) & 1:
                    grid[r0 + s, bb] = T[r0 + (s | 1 << bb)] - T[r0 + s]
    L = P.compose(grid, b)
    for k in range(4):
        r0, r1 = b.row_off[k], b.row_off[k + 1]
        np.testing.assert_allclose(L[r0:r1], T[r0:r1] - T[r0], atol=1e-12)


def test_compose_three_bits_by_hand():
    b, _ = small_batch([3])
    g = np.random.default_rng(13).normal(size=(8, 3))
    for s in range(8):
        for bb in range(3):
            if (s >> bb) & 1:
                g[s, bb] = np.nan
    L = P.compose(g, b)
    assert L[0] == 0
    assert L[0b001] == g[0, 0] and L[0b010] == g[0, 1] and L[0b100] == g[0, 2]
    assert L[0b011] == g[0, 0] + g[0b001, 1]
    assert L[0b101] == g[0, 0] + g[0b001, 2]
    assert L[0b110] == g[0, 1] + g[0b010, 2]
    assert L[0b111] == g[0, 0] + g[0b001, 1] + g[0b011, 2]


# ---------------------------------------------------------------- rank ----
def _selection_rank(s, tau, n, first):
    """Brute force: repeatedly take the best remaining candidate."""
    left = [i for i in range(first, len(s)) if s[i] > tau]
    out = []
    while left and len(out) < n:
        best = left[0]
        for i in left[1:]:
            if s[i] > s[best] or (s[i] == s[best] and i < best):
                best = i
        out.append(best)
        left.remove(best)
    return out


def test_rank_matches_selection_bruteforce():
    rng = np.random.default_rng(14)
    for trial in range(300):
        m = int(rng.integers(0, 12))
        s = np.round(rng.normal(0.05, 0.1, size=m), 2)   # rounding creates ties
        if trial % 7 == 0 and m:
            s[rng.integers(0, m)] = np.nan
        n = int(rng.integers(1, 6))
        first = int(rng.integers(0, 2))
        got = [i for i, _ in P.rank(s, P.TAU, n, first)]
        assert got == _selection_rank(s, P.TAU, n, first)


def test_rank_permutation_threshold_monotone_and_prefix():
    rng = np.random.default_rng(15)
    s = rng.normal(0, 0.1, size=64)
    full = [i for i, _ in P.rank(s, -np.inf, 10 ** 9, first=1)]
    assert sorted(full) == list(range(1, 64))
    taus = np.sort(rng.normal(0, 0.1, size=6))
    outs = [[i for i, _ in P.rank(s, t, 10 ** 9, 1)] for t in taus]
    for a, b in zip(outs[:-1], outs[1:]):
        assert a[:len(b)] == b
    for t in taus:
        out = P.rank(s, t, 10 ** 9, 1)
        assert all(v > t for _, v in out)
        assert all(out[i][1] >= out[i + 1][1] for i in range(len(out) - 1))
    assert [i for i, _ in P.rank(s, 0.0, 2, 1)] == [i for i, _ in P.rank(s, 0.0, 5, 1)][:2]


def test_threshold_is_five_percent():
    assert abs(math.exp(P.TAU) - 1.05) < 1e-15


# ------------------------------------------------------------- checker ----
def test_checker_accepts_ties_and_rejects_errors():
    s = np.array([0.0, 0.30, 0.20, 0.2000001, 0.10, 0.0488])
    tol = 1e-5
    assert check_list([1, 2, 3], [0.3, 0.2, 0.2000001], s, P.TAU, 3, tol, first=1) == []
    assert check_list([1, 3, 2], [0.3, 0.2000001, 0.2], s, P.TAU, 3, tol, first=1) == []
    assert check_list([1, 2, 4], [0.3, 0.2, 0.1], s, P.TAU, 3, tol, first=1) != []
    assert check_list([2, 1, 3], [0.2, 0.3, 0.2], s, P.TAU, 3, tol, first=1) != []
    assert check_list([1, 2], [0.3, 0.2], s, P.TAU, 3, tol, first=1) != []
    assert check_list([1, 2, 3], [0.3, 0.21, 0.2], s, P.TAU, 3, tol, first=1) != []
    # near the threshold either answer is accepted
    s2 = np.array([0.0, 0.3, P.TAU + 1e-7])
    assert check_list([1], [0.3], s2, P.TAU, 3, tol, first=1) == []
    assert check_list([1, 2], [0.3, P.TAU], s2, P.TAU, 3, tol, first=1) == []


# ------------------------------------------------------- whole method ----
def test_fit_counts_and_untrained():
    b, D = small_batch([3, 2, 4], E=6)
    m = P.fit(b, D)
    opt, *_ = P.candidate_pairs(b.nopts, b.opt_ids, b.opt_off, b.row_off)
    for o in range(D):
        assert m["counts"][o] == (opt == o).sum()
        assert np.isnan(m["W"][o]).all() == (m["counts"][o] == 0)


def test_loko_fold_structure():
    from synthgen import make_batch
    b = make_batch(1910, range(2), 40, 6, dtype=np.float64)
    folds = P.leave_one_kernel_out(b, 6)
    assert len(folds) == 2
    for f in folds:
        assert (f["model"]["counts"] == 32).all()
        assert len(f["suggestions"]) == 1
        assert len(f["suggestions"][0]) <= 3
        assert f["table"][0] == 0.0
