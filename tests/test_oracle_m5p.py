"""Pins of the M5P model-tree oracle: the split against a brute force over
every threshold with the standard deviations taken directly, trees whose
answer is known (a step, a piecewise-linear function, a linear function, a
constant), the smoothing recursion in closed form, a hand-worked error
estimate, and structural invariants."""
import numpy as np
import pytest

from oracle import m5p as M
from synthgen import make_batch


def _route_counts(tree, Z):
    counts = np.zeros(len(tree["feat"]), dtype=np.int64)
    for z in Z:
        i = 0
        counts[i] += 1
        while tree["feat"][i] >= 0:
            i = tree["left"][i] if z[tree["feat"][i]] <= tree["thr"][i] else tree["right"][i]
            counts[i] += 1
    return counts


def test_split_is_the_brute_force_argmax():
    rng = np.random.default_rng(5)
    for trial in range(20):
        n, E = int(rng.integers(8, 16)), 3
        Z = rng.normal(size=(n, E))
        if trial % 3 == 0:
            Z[:, 1] = np.round(Z[:, 1])          # repeated values: fewer admissible thresholds
        y = rng.normal(size=n) + Z[:, 0] ** 2
        best, arg = -np.inf, None
        for j in range(E):
            vals = np.unique(Z[:, j])
            for a, b in zip(vals[:-1], vals[1:]):
                t = 0.5 * (a + b)
                left = Z[:, j] <= t
                if left.sum() < M.MIN_LEAF or (~left).sum() < M.MIN_LEAF:
                    continue
                sdr = np.std(y) - left.mean() * np.std(y[left]) - (~left).mean() * np.std(y[~left])
                if sdr > best:
                    best, arg = sdr, (j, t)
        got = M.best_split(Z, y, M.MIN_LEAF, 0.0)
        if arg is None:
            assert got is None
            continue
        assert (got[0], got[1]) == arg
        assert abs(got[2] - best) < 1e-12


def test_hand_worked_error_estimate():
    # constant model on y = [0, 0, 0, 0, 4]: mean 0.8, mean |residual| 6.4 / 5
    # = 1.28, v = 1 parameter, factor (5 + 1) / (5 - 1) = 1.5
    m = M.fit_node_model(np.zeros((5, 2)), np.array([0, 0, 0, 0, 4.0]), [])
    assert abs(m["b"] - 0.8) < 1e-15 and abs(m["est"] - 1.92) < 1e-12
    # v >= n: no estimate
    assert M.fit_node_model(np.eye(3), np.ones(3), [0, 1])["est"] == np.inf


def test_step_function_splits_once_and_smooths_in_closed_form():
    rng = np.random.default_rng(6)
    Z = rng.normal(size=(200, 5))
    y = np.where(Z[:, 3] > 0.2, 1.0, -1.0)
    tree = M.build(Z, y)
    lo, hi = Z[Z[:, 3] <= 0.2, 3].max(), Z[Z[:, 3] > 0.2, 3].min()
    assert list(tree["feat"]) == [3, -1, -1] and list(tree["left"]) == [1, -1, -1]
    assert abs(tree["thr"][0] - 0.5 * (lo + hi)) < 1e-15
    for z, t in zip(Z, y):
        assert M.predict_one(tree, z, 0.0)[0] == pytest.approx(t, abs=1e-12)
    # smoothing: (n_c * leaf + 15 * root model) / (n_c + 15); the root model
    # uses feature 3 only and is the simple regression line of y on z_3
    x = Z[:, 3]
    slope = np.sum((x - x.mean()) * (y - y.mean())) / np.sum((x - x.mean()) ** 2)
    icpt = y.mean() - slope * x.mean()
    n_hi = int((x > 0.2).sum())
    for z, t in zip(Z[:20], y[:20]):
        nc = n_hi if t > 0 else 200 - n_hi
        want = (nc * t + 15 * (slope * z[3] + icpt)) / (nc + 15)
        assert M.predict_one(tree, z)[0] == pytest.approx(want, abs=1e-12)


def test_piecewise_linear_is_recovered_exactly_without_smoothing():
    rng = np.random.default_rng(7)
    Z = rng.normal(size=(400, 4))
    y = 2 * Z[:, 0] + np.where(Z[:, 1] > 0, 3.0, -3.0)
    tree = M.build(Z, y)
    assert tree["feat"][0] == 1 and len(tree["feat"]) == 3       # the step, then exact leaf models
    for z, t in zip(Z, y):
        assert M.predict_one(tree, z, 0.0)[0] == pytest.approx(t, abs=1e-9)


def test_linear_function_prunes_to_one_exact_model():
    rng = np.random.default_rng(8)
    Z = rng.normal(size=(300, 5))
    y = 3 * Z[:, 0] + 1
    tree = M.build(Z, y)
    assert len(tree["feat"]) == 1
    m = tree["model"][0]
    assert m["A"] == [0] and m["w"][0] == pytest.approx(3, abs=1e-10) and m["b"] == pytest.approx(1, abs=1e-10)
    for z, t in zip(Z[:50], y[:50]):
        assert M.predict_one(tree, z)[0] == pytest.approx(t, abs=1e-9)


def test_degenerate_inputs_give_one_leaf():
    rng = np.random.default_rng(9)
    Z = rng.normal(size=(50, 3))
    tree = M.build(Z, np.full(50, 0.25))                       # constant labels
    assert len(tree["feat"]) == 1 and M.predict_one(tree, Z[0])[0] == pytest.approx(0.25, abs=1e-15)
    y = rng.normal(size=7)                                     # fewer than 2 * MIN_LEAF cases
    tree = M.build(Z[:7], y)
    assert len(tree["feat"]) == 1 and tree["model"][0]["A"] == []
    assert M.predict_one(tree, Z[0])[0] == pytest.approx(y.mean(), abs=1e-15)


def test_structure_invariants_on_noisy_data():
    rng = np.random.default_rng(10)
    Z = rng.normal(size=(600, 6))
    y = np.sin(2 * Z[:, 0]) + 0.5 * np.abs(Z[:, 2]) + 0.1 * rng.normal(size=600)
    tree = M.build(Z, y)
    assert len(tree["feat"]) > 1
    assert np.array_equal(_route_counts(tree, Z), tree["n"])
    for i, f in enumerate(tree["feat"]):
        if f >= 0:
            L, R = tree["left"][i], tree["right"][i]
            assert L == i + 1 and R > L                            # preorder
            assert tree["n"][L] + tree["n"][R] == tree["n"][i]
            assert set(tree["model"][i]["A"]) >= {f}
        else:
            assert tree["n"][i] >= M.MIN_LEAF and tree["left"][i] == tree["right"][i] == -1
    # without smoothing a prediction is the leaf model's value
    for z in Z[:30]:
        i = 0
        while tree["feat"][i] >= 0:
            i = tree["left"][i] if z[tree["feat"][i]] <= tree["thr"][i] else tree["right"][i]
        assert M.predict_one(tree, z, 0.0)[0] == pytest.approx(M.model_value(tree["model"][i], z), abs=1e-15)


def test_fit_and_run_on_a_synthetic_batch():
    tr = make_batch(12, range(100, 124), 16, 4)
    te = make_batch(12, range(6), 16, 4, brange=(0, 4))
    model = M.fit(tr, 4)
    assert sorted(model["trees"]) == [0, 1, 2, 3]
    for t in model["trees"].values():
        assert t["n"][0] == 24 * 8
    grid, table, res = M.run(model, te)
    assert np.isfinite(table).all() and len(res) == te.K
    _, margin = M.predict_grid(model, te)
    assert (margin > 0).all()


def test_collinear_features_are_dropped_in_order():
    # z1 = 2 z0 exactly and z2 constant: only z0 of A = [0, 1, 2] is kept, so
    # y = 3 z0 + 1 is fitted by w = (3, 0, 0), b = 1, with two parameters
    rng = np.random.default_rng(11)
    z0 = rng.normal(size=40)
    Z = np.stack([z0, 2 * z0, np.full(40, 0.7)], axis=1)
    y = 3 * z0 + 1
    assert M.independent_features(Z, [0, 1, 2]) == [0]
    assert M.independent_features(Z, [1, 0]) == [1]
    m = M.fit_node_model(Z, y, [0, 1, 2])
    np.testing.assert_allclose(m["w"], [3, 0, 0], atol=1e-12)
    assert abs(m["b"] - 1) < 1e-12 and m["est"] < 1e-12
    # an independent third column is kept
    Z[:, 2] = rng.normal(size=40)
    assert M.independent_features(Z, [0, 1, 2]) == [0, 2]
