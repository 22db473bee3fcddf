"""Pins of the IBK oracle: neighbour search against scipy's k-d tree (an
independent search), a hand-worked 1-D case, the tie rule, k = 1 reproducing
the training labels exactly (so the composed table telescopes to the measured
log-speedups), and invariance under a rotation of the feature space."""
import numpy as np
from scipy.spatial import cKDTree

from oracle import knn as N
from oracle import plain as P
from synthgen import make_batch


def test_neighbours_match_a_kd_tree():
    rng = np.random.default_rng(1)
    Z = rng.normal(size=(500, 16))
    tree = cKDTree(Z)
    for q in rng.normal(size=(40, 16)):
        idx, d2 = N.neighbours(Z, q, 10)
        dt, it = tree.query(q, k=10)
        np.testing.assert_allclose(np.sqrt(d2), dt, rtol=1e-12)
        assert list(idx) == list(it)
        assert np.all(np.diff(d2) >= 0)


def test_hand_worked_one_dimensional_case():
    db = {"Z": {0: np.array([[0.0], [1.0], [3.0], [6.0]])}, "y": {0: np.array([1.0, 2.0, 3.0, 4.0])}}
    # distances to 2.2: 2.2, 1.2, 0.8, 3.8 -> nearest two are samples 2 and 1
    idx, d2 = N.neighbours(db["Z"][0], np.array([2.2]), 2)
    assert list(idx) == [2, 1]
    np.testing.assert_allclose(d2, [0.64, 1.44])
    assert N.predict_one(db, np.array([2.2]), 0, k=2) == 2.5
    assert N.predict_one(db, np.array([2.2]), 0, k=10) == 2.5       # fewer than k samples: all
    assert N.predict_one(db, np.array([-5.0]), 0, k=1) == 1.0


def test_equal_distances_keep_the_first_stored_sample():
    Z = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 0.0], [-1.0, 0.0]])
    assert list(N.neighbours(Z, np.array([1.0, 0.0]), 1)[0]) == [0]
    assert list(N.neighbours(Z, np.array([1.0, 0.0]), 2)[0]) == [0, 2]
    # the origin is equidistant from all four
    assert list(N.neighbours(Z, np.zeros(2), 3)[0]) == [0, 1, 2]


def test_one_neighbour_reproduces_the_training_labels():
    tr = make_batch(5, range(12), 24, 5, brange=(1, 5))
    db = N.database(tr, 5)
    grid, table, _ = N.run(db, tr, k=1)
    opt, before, after, kern, S, b = P.candidate_pairs(tr.nopts, tr.opt_ids, tr.opt_off, tr.row_off)
    y = P.pair_labels(tr.cycles, before, after)
    np.testing.assert_array_equal(grid[before, b], y)
    # composing measured steps telescopes to ln cyc(baseline) - ln cyc(S)
    for k in range(len(tr.nopts)):
        r0, r1 = tr.row_off[k], tr.row_off[k + 1]
        want = np.log(tr.cycles[r0].astype(np.float64)) - np.log(tr.cycles[r0:r1].astype(np.float64))
        np.testing.assert_allclose(table[r0:r1], want, atol=1e-12)


def test_database_holds_every_pair_once():
    tr = make_batch(6, range(20), 16, 6, brange=(0, 6))
    db = N.database(tr, 6)
    for o in range(6):
        want = sum(1 << (int(tr.nopts[k]) - 1) for k in range(len(tr.nopts))
                   if o in tr.opt_ids[tr.opt_off[k]:tr.opt_off[k + 1]])
        assert (db["Z"][o].shape[0] if o in db["Z"] else 0) == want


def test_rotation_invariance():
    rng = np.random.default_rng(3)
    Z = rng.normal(size=(300, 8))
    y = rng.normal(size=300)
    Q, _ = np.linalg.qr(rng.normal(size=(8, 8)))
    a = {"Z": {0: Z}, "y": {0: y}}
    b = {"Z": {0: Z @ Q}, "y": {0: y}}
    for q in rng.normal(size=(30, 8)):
        assert abs(N.predict_one(a, q, 0) - N.predict_one(b, q @ Q, 0)) < 1e-12
