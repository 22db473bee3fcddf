"""Pins of the all-paths composition and the greedy re-profiling oracle:
the level recursion against a brute force over every ordering, telescoping
on exact step tables, hand-worked 2-bit cases, greedy properties."""
import numpy as np

from oracle import paths as A
from oracle import plain as P
from synthgen import make_batch

TAU = P.TAU
NAN = np.nan


class _One:
    """A batch of one kernel with B optimisations (the layout fields only)."""
    def __init__(self, B):
        self.nopts = np.array([B])
        self.row_off = np.array([0, 1 << B])


def _grid(rng, B):
    g = rng.normal(0.05, 0.15, ((1 << B), B))
    for S in range(1 << B):
        for b in range(B):
            if (S >> b) & 1:
                g[S, b] = np.nan
    return g


def test_level_recursion_equals_the_mean_over_orderings():
    rng = np.random.default_rng(1)
    for B in (1, 2, 3, 4):
        for _ in range(5):
            g = _grid(rng, B)
            t = A.compose_allpaths(g, _One(B))
            for S in range(1 << B):
                assert abs(t[S] - A.allpaths_by_orderings(g, S)) < 1e-12


def test_exact_step_table_telescopes():
    rng = np.random.default_rng(2)
    B = 5
    T = rng.normal(0, 0.3, 1 << B)
    g = np.full((1 << B, B), np.nan)
    for S in range(1 << B):
        for b in range(B):
            if not (S >> b) & 1:
                g[S, b] = T[S | (1 << b)] - T[S]
    np.testing.assert_allclose(A.compose_allpaths(g, _One(B)), T - T[0], atol=1e-12)


def test_hand_worked_two_bits():
    g = np.array([[0.1, 0.2], [NAN, 0.4], [0.5, NAN], [NAN, NAN]])
    t = A.compose_allpaths(g, _One(2))
    # L(1) = P(0,0); L(2) = P(0,1); L(3) = ((0.2 + 0.5) + (0.1 + 0.4)) / 2
    np.testing.assert_allclose(t, [0.0, 0.1, 0.2, 0.6], atol=1e-15)
    # the ascending chain gives P(0,0) + P(1,1) = 0.5 instead
    assert abs(P.compose(g, _One(2))[3] - 0.5) < 1e-15


def test_greedy_hand_worked():
    g = np.array([[0.1, 0.2], [NAN, 0.4], [0.5, NAN], [NAN, NAN]])
    path, steps = A.greedy_kernel(g, 2, TAU)
    assert path == [0, 2, 3] and np.allclose(steps, [0.2, 0.5])
    g2 = g.copy()
    g2[2, 0] = 0.01                                   # below the threshold: stop
    assert A.greedy_kernel(g2, 2, TAU) == ([0, 2], [0.2])
    g3 = g.copy()
    g3[0] = [0.2, 0.2]                                # tie: the smaller bit
    assert A.greedy_kernel(g3, 2, TAU)[0][:2] == [0, 1]
    g4 = g.copy()
    g4[0] = [0.01, -0.3]                              # nothing above the threshold
    assert A.greedy_kernel(g4, 2, TAU) == ([0], [])


def test_greedy_properties():
    rng = np.random.default_rng(3)
    for B in (1, 3, 6):
        for _ in range(20):
            g = _grid(rng, B)
            path, steps = A.greedy_kernel(g, B, TAU)
            assert path[0] == 0 and len(path) == len(steps) + 1 <= B + 1
            for i, v in enumerate(steps):
                S, S2 = path[i], path[i + 1]
                b = (S2 ^ S).bit_length() - 1
                assert S2 == S | (1 << b) and not (S >> b) & 1
                assert v == g[S, b] and v > TAU
                assert v == max(g[S, c] for c in range(B) if not (S >> c) & 1)
            last = path[-1]
            assert all(g[last, c] <= TAU for c in range(B) if not (last >> c) & 1)


def test_allpaths_on_a_fitted_model_is_finite_and_zero_at_baseline():
    tr = make_batch(8, range(100, 140), 16, 5, brange=(1, 5))
    te = make_batch(8, range(20), 16, 5, brange=(0, 5))
    model = P.fit(tr, 5)
    grid = P.predict_grid(model, te)
    t = A.compose_allpaths(grid, te)
    assert np.isfinite(t).all()
    assert (t[te.row_off[:-1]] == 0).all()
