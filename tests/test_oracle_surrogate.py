"""Pins of the FP64 surrogate oracle: closed-form GELU values, finite
differences of the hand-written backward, Adam's first step, bfloat16
rounding.  CPU only."""
import math

import numpy as np
import pytest

from oracle import surrogate as M


def test_gelu_closed_form_values():
    # gelu(t) = t * Phi(t), Phi the standard normal CDF
    assert M.gelu(0.0) == 0.0
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(-1.0) + 0.15865525393145707) < 1e-15
    assert abs(M.gelu(2.0) - 2 * 0.9772498680518208) < 1e-15
    assert abs(M.gelu_grad(0.0) - 0.5) < 1e-15
    assert abs(M.gelu(12.0) - 12.0) < 1e-12 and abs(M.gelu(-12.0)) < 1e-12
    assert abs(M.gelu_grad(12.0) - 1.0) < 1e-12


def test_gelu_grad_finite_difference():
    t = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (M.gelu(t + h) - M.gelu(t - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(t), fd, rtol=0, atol=1e-9)


@pytest.mark.parametrize("sizes", [(8, 16, 16, 4), (5, 7, 3)])
def test_backward_matches_central_differences(sizes):
    rng = np.random.default_rng(21)
    params = M.init_params(rng, sizes)
    x = rng.normal(size=(6, sizes[0]))
    tgt = rng.normal(size=(6, sizes[-1]))

    def loss(ps):
        return M.mse(M.forward(ps, x)[0], tgt)[0]

    y, cache = M.forward(params, x)
    _, dy = M.mse(y, tgt)
    grads = M.backward(params, cache, dy)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for j, arr in enumerate((W, b)):
            g = grads[li][j]
            flat = arr.reshape(-1)
            for idx in range(flat.size):
                old = flat[idx]
                flat[idx] = old + h
                lp = loss(params)
                flat[idx] = old - h
                lm = loss(params)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                gv = g.reshape(-1)[idx]
                assert abs(gv - fd) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (li, j, idx, gv, fd)


def test_zero_first_layer_makes_output_constant():
    rng = np.random.default_rng(22)
    params = M.init_params(rng, (8, 16, 16, 4))
    params[0] = (np.zeros((8, 16)), np.zeros(16))
    x = rng.normal(size=(5, 8))
    y, _ = M.forward(params, x)
    W2, b2 = params[1]
    W3, b3 = params[2]
    want = M.gelu(b2) @ W3 + b3
    np.testing.assert_allclose(y, np.broadcast_to(want, y.shape), atol=1e-14)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(23)
    params = M.init_params(rng, (4, 6, 3))
    grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
    st = M.adam_init(params)
    new = M.adam_step(params, grads, st, lr=1e-3)
    for (W, b), (nW, nb), (gW, gb) in zip(params, new, grads):
        np.testing.assert_allclose(nW - W, -1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-10)
        np.testing.assert_allclose(nb - b, -1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-10)
    assert st["t"] == 1


def test_adam_overfits_a_tiny_batch():
    rng = np.random.default_rng(24)
    params = M.init_params(rng, (6, 32, 32, 3))
    x = rng.normal(size=(8, 6))
    tgt = rng.normal(0, 0.3, size=(8, 3))
    st = M.adam_init(params)
    first = None
    for _ in range(1500):
        y, cache = M.forward(params, x)
        l, dy = M.mse(y, tgt)
        first = l if first is None else first
        params = M.adam_step(params, M.backward(params, cache, dy), st, lr=3e-3)
    assert l < 1e-4 * first


def test_bf16_round_ties_to_even():
    assert M.bf16_round(1.0) == 1.0
    assert M.bf16_round(1 + 2 ** -8) == 1.0                  # halfway, even mantissa below
    assert M.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6      # halfway, rounds up to even
    assert M.bf16_round(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert M.bf16_round(3.14159) == 3.140625
    assert M.bf16_round(-2.0 ** -130) == -2.0 ** -130        # subnormal kept exactly
    assert math.isnan(M.bf16_round(np.nan))
