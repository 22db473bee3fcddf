"""Pins of the serving rule's oracle: hand-worked cases on 2-bit kernels and
properties that hold for any tables (a perfect surrogate answers exactly as
the plain method; a surrogate off by more than the tolerance never answers)."""
import numpy as np

from oracle import plain as P
from oracle import serve as V

TAU = P.TAU


def test_hand_worked_two_bit_kernel():
    # surrogate list: S=3 (0.30), S=1 (0.20); n=3 so the list is short and
    # S=2 (0.01 >= tau - 0.1 = -0.0512) is in the band; every difference
    # (0.02, 0.05, 0.01) is within 0.1: the surrogate answers, plain values
    sur = [0.0, 0.20, 0.01, 0.30]
    fb, ans, judged = V.serve_kernel(sur, [0.0, 0.25, 0.02, 0.28], n=3)
    assert not fb and judged == [3, 1, 2]
    assert ans == [(3, 0.28), (1, 0.25)]
    # the band catches a subset the surrogate's threshold dropped: plain 0.15
    fb, ans, _ = V.serve_kernel(sur, [0.0, 0.25, 0.15, 0.28], n=3)
    assert fb and ans == [(3, 0.28), (1, 0.25), (2, 0.15)]
    # with n=2 the list is full: no band, S=2 is not judged
    fb, ans, judged = V.serve_kernel(sur, [0.0, 0.25, 0.15, 0.28], n=2)
    assert not fb and judged == [3, 1] and ans == [(3, 0.28), (1, 0.25)]
    # a listed subset off by more than the tolerance
    fb, ans, _ = V.serve_kernel(sur, [0.0, 0.31, 0.02, 0.28], n=3)
    assert fb and ans == [(1, 0.31), (3, 0.28)]
    # band larger than the cap
    fb, _, _ = V.serve_kernel(sur, [0.0, 0.25, 0.02, 0.28], n=3, cap=0)
    assert fb
    # a non-finite plain value on a judged subset
    fb, _, _ = V.serve_kernel(sur, [0.0, 0.25, np.nan, 0.28], n=3)
    assert fb


def test_kept_answer_obeys_the_threshold_and_the_plain_order():
    """Tier 3's contract on a kept answer (Section 2: only choices above the
    threshold, sorted by expected benefit), by the plain values: a threshold
    breach falls back, the order is restored by sorting."""
    # S=3 is listed (surrogate 0.12) and within the tolerance of its plain
    # value 0.048, which is not above tau = 0.04879: fall back
    fb, ans, _ = V.serve_kernel([0.0, 0.20, 0.01, 0.12], [0.0, 0.25, 0.02, 0.048], n=3)
    assert fb and ans == [(1, 0.25)]
    # the same with plain 0.049 (above tau): kept
    fb, ans, _ = V.serve_kernel([0.0, 0.20, 0.01, 0.12], [0.0, 0.25, 0.02, 0.049], n=3)
    assert not fb and ans == [(1, 0.25), (3, 0.049)]
    # listed 3 before 1, but the plain values order them 1 before 3: kept,
    # in the plain order
    fb, ans, _ = V.serve_kernel([0.0, 0.20, 0.01, 0.30], [0.0, 0.29, 0.02, 0.22], n=3)
    assert not fb and ans == [(1, 0.29), (3, 0.22)]
    # equal plain values: the smaller subset first
    fb, ans, _ = V.serve_kernel([0.0, 0.20, 0.01, 0.30], [0.0, 0.25, 0.02, 0.25], n=3)
    assert not fb and ans == [(1, 0.25), (3, 0.25)]
    # a band subset (S=2, surrogate 0.01) whose plain value 0.06 is above tau
    fb, ans, _ = V.serve_kernel([0.0, 0.20, 0.01, 0.30], [0.0, 0.25, 0.06, 0.28], n=3)
    assert fb and ans == [(3, 0.28), (1, 0.25), (2, 0.06)]


def test_band_is_below_threshold_and_ascending():
    sur = [0.0, -0.06, 0.0, 0.04, 0.2, -0.2, 0.03, 0.049]
    listed = [S for S, _ in P.rank(sur, TAU, 3, first=1)]
    assert listed == [4, 7]                       # 0.049 > tau = 0.04879...
    assert V.band(sur, listed, TAU, 3, 0.1) == [2, 3, 6]   # >= -0.0512, not listed
    assert V.band(sur, listed, TAU, 2, 0.1) == []          # full list: no band


def _tables(rng, K, B):
    return [np.concatenate([[0.0], rng.normal(0.05, 0.15, (1 << B) - 1)]) for _ in range(K)]


def test_perfect_surrogate_answers_as_the_plain_method():
    rng = np.random.default_rng(1)
    for B in (1, 3, 6):
        for t in _tables(rng, 50, B):
            fb, ans, judged = V.serve_kernel(t, t, cap=1 << B)
            assert not fb
            assert ans == P.rank(t, TAU, 3, first=1)


def test_surrogate_off_by_more_than_tol_never_answers():
    rng = np.random.default_rng(2)
    for t in _tables(rng, 100, 5):
        sur = t + 0.5
        sur[0] = 0.0
        fb, ans, judged = V.serve_kernel(sur, t, cap=64)
        assert fb == bool(judged)
        if fb:
            assert ans == P.rank(t, TAU, 3, first=1)


def test_kept_answers_are_confirmed_by_the_plain_values():
    rng = np.random.default_rng(3)
    kept = 0
    for t in _tables(rng, 300, 6):
        sur = t + rng.normal(0, 0.04, t.shape)
        sur[0] = 0.0
        fb, ans, judged = V.serve_kernel(sur, t)
        listed = [S for S, _ in P.rank(sur, TAU, 3, first=1)]
        if fb:
            assert ans == P.rank(t, TAU, 3, first=1)
        else:
            kept += 1
            assert sorted(S for S, _ in ans) == sorted(listed)
            assert all(abs(sur[S] - t[S]) <= 0.1 and v == t[S] for S, v in ans)
            assert set(listed) <= set(judged)
            # the kept answer is Tier 3's ranking of the plain values over the judged subsets
            sub = np.full(t.shape, -np.inf)
            sub[judged] = t[judged]
            assert ans == P.rank(sub, TAU, 3, first=1)
    assert kept > 0
