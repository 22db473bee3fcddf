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


def test_adam_constant_gradient_steps_lr_every_step():
    """With a constant gradient g, the moments after t steps are
    (1 - beta1^t) g and (1 - beta2^t) g^2, so the bias-corrected estimates are
    g and g^2 at every step and each update moves a parameter by exactly
    -lr g / (|g| + eps): a bias correction with the wrong power of beta at
    t >= 2 would shrink or grow these steps."""
    params = [(np.array([[0.25, -1.5]]), np.array([3.0]))]
    g = [(np.array([[0.3, -2.0]]), np.array([1e-3]))]
    st = M.adam_init(params)
    p = params
    for t in range(1, 7):
        new = M.adam_step(p, g, st, lr=1e-2)
        for (W, b), (nW, nb), (gW, gb) in zip(p, new, g):
            np.testing.assert_allclose(nW - W, -1e-2 * gW / (np.abs(gW) + 1e-8), rtol=1e-9)
            np.testing.assert_allclose(nb - b, -1e-2 * gb / (np.abs(gb) + 1e-8), rtol=1e-9)
        p = new
        assert st["t"] == t


def test_adam_three_steps_hand_worked():
    """Gradients 1, -1, 2 on one parameter (beta 0.9 / 0.999, lr 1e-3,
    eps 1e-8), worked by hand in exact fractions:
      t=1: m = 1/10,      v = 1/1000;           m/(1-0.9)   = 1,       v/(1-0.999)     = 1
      t=2: m = -1/100,    v = 1999/10^6;        m/(1-0.81)  = -1/19,   v/(1-0.998001)  = 1
      t=3: m = 191/1000,  v = 5997001/10^9;     m/(1-0.729) = 191/271, v/(1-0.997002999) = 5997001/2997001
    so the parameter moves by -1e-3 * 1/(1 + 1e-8), then +1e-3 * (1/19)/(1 + 1e-8),
    then -1e-3 * (191/271)/(sqrt(5997001/2997001) + 1e-8)."""
    steps = [-1e-3 * 1.0 / (1.0 + 1e-8),
             1e-3 * (1.0 / 19.0) / (1.0 + 1e-8),
             -1e-3 * (191.0 / 271.0) / (math.sqrt(5997001.0 / 2997001.0) + 1e-8)]
    p = [(np.array([[0.5]]), np.array([0.0]))]
    st = M.adam_init(p)
    want = 0.5
    for g, d in zip((1.0, -1.0, 2.0), steps):
        p = M.adam_step(p, [(np.array([[g]]), np.array([0.0]))], st, lr=1e-3)
        want += d
        assert abs(p[0][0][0, 0] - want) <= 1e-15, (st["t"], p[0][0][0, 0], want)
    # the second and third moments by themselves
    assert abs(st["m"][0][0][0, 0] - 0.191) <= 1e-16
    assert abs(st["v"][0][0][0, 0] - 5997001e-9) <= 2e-17


def test_backward_full_size_network_sampled_central_differences():
    """The 128 -> 512 -> 512 -> 64 network itself: the hand-written
    gradient of 24 sampled coordinates (four of every weight and bias
    tensor, including the largest-gradient entry of each) against FP64
    central differences, h = 1e-6."""
    rng = np.random.default_rng(31)
    params = M.init_params(rng, (128, 512, 512, 64))
    x = rng.normal(size=(4, 128))
    tgt = rng.normal(0.1, 0.3, size=(4, 64))

    def loss(ps):
        return M.mse(M.forward(ps, x)[0], tgt)[0]

    y, cache = M.forward(params, x)
    _, dy = M.mse(y, tgt)
    grads = M.backward(params, cache, dy)
    h = 1e-6
    checked = 0
    for li in range(3):
        for j in range(2):
            arr, g = params[li][j], grads[li][j]
            flat, gf = arr.reshape(-1), g.reshape(-1)
            picks = [int(np.argmax(np.abs(gf)))] + [int(i) for i in rng.choice(flat.size, 3, replace=False)]
            for idx in picks:
                old = flat[idx]
                flat[idx] = old + h
                lp = loss(params)
                flat[idx] = old - h
                lm = loss(params)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(gf[idx] - fd) <= 1e-6 * abs(fd) + 1e-10, (li, j, idx, gf[idx], fd)
                checked += 1
    assert checked == 24
