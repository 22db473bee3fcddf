"""GPU surrogate MLP (BF16 matrix cores, hand-written backward, Adam) against
the FP64 oracle evaluated at the same BF16 rounding points (weights, input and
hidden activations rounded to bfloat16).  Tolerance 3e-2 relative for BF16
results (max abs error over max abs value, per tensor); FP32 Adam 1e-5."""
import numpy as np
import pytest
import torch

from oracle import surrogate as M

pytestmark = pytest.mark.gpu

BF16_RTOL = 3e-2


@pytest.fixture(scope="module")
def S():
    from paper_1910_07776_amd import plain, surrogate
    return plain, surrogate


@pytest.fixture(scope="module")
def ctx(S):
    c = S[0].Context(0)
    yield c
    c.close()


def oracle_params(mlp, flat):
    """GPU layout (W [out x in]) -> oracle layout (W [in x out])."""
    u = mlp.unflatten(np.asarray(flat, dtype=np.float64))
    return [(u["W1"].T, u["b1"]), (u["W2"].T, u["b2"]), (u["W3"].T, u["b3"])]


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def batch(B, n_in, n_out, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, size=(B, n_in)).astype(np.float32)
    t = rng.normal(0.1, 0.3, size=(B, n_out)).astype(np.float32)
    return x, t


@pytest.mark.parametrize("dims,B", [((128, 512, 64), 300), ((32, 64, 16), 37), ((128, 512, 1024), 129)])
def test_forward_and_loss_match_oracle(S, ctx, dims, B):
    plain, sur = S
    mlp = sur.MLP(ctx, *dims, max_batch=512, seed=3)
    x, t = batch(B, dims[0], dims[2], 1)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = mlp(xd)
    op = oracle_params(mlp, mlp.params.cpu().numpy())
    yo, _ = M.forward_bf16(op, x)
    assert rel(y.cpu().numpy(), yo) < BF16_RTOL
    yl = torch.empty_like(y)
    loss = mlp.loss_raw(xd, td, y=yl)
    torch.cuda.synchronize()
    assert torch.equal(yl, y)
    lo, _ = M.mse(yo, t)
    assert abs(float(loss.item()) - lo) <= BF16_RTOL * lo
    mlp.close()


@pytest.mark.parametrize("dims,B", [((128, 512, 64), 256), ((32, 64, 16), 45)])
def test_backward_matches_oracle_gradient(S, ctx, dims, B):
    plain, sur = S
    mlp = sur.MLP(ctx, *dims, max_batch=512, seed=4)
    x, t = batch(B, dims[0], dims[2], 2)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    mlp.loss_raw(xd, td)
    g = mlp.backward_raw(mlp.params, None, B, torch.empty_like(mlp.params))
    op = oracle_params(mlp, mlp.params.cpu().numpy())
    pr = [(M.bf16_round(W), b) for W, b in op]
    y, cache = M.forward(pr, M.bf16_round(x), round_hidden=M.bf16_round)
    _, dy = M.mse(y, t)
    go = M.backward(pr, cache, dy)
    gu = mlp.unflatten(g.cpu().numpy().astype(np.float64))
    for li, (Wn, bn) in enumerate((("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
        assert rel(gu[Wn], go[li][0].T) < BF16_RTOL, Wn
        assert rel(gu[bn], go[li][1]) < BF16_RTOL, bn
    # the same through torch.autograd with an explicit output gradient
    p = mlp.params.clone().requires_grad_(True)
    yy = sur.SurrogateFn.apply(xd, p, mlp)
    ((yy - td) ** 2).mean().backward()
    torch.cuda.synchronize()
    assert rel(p.grad.cpu().numpy(), g.cpu().numpy()) < 1e-2
    mlp.close()


def test_adam_matches_oracle(S, ctx):
    plain, sur = S
    mlp = sur.MLP(ctx, 32, 64, 16, max_batch=64, seed=5)
    rng = np.random.default_rng(6)
    p0 = mlp.params.cpu().numpy().astype(np.float64)
    op = [(p0, np.zeros(1))]
    st = M.adam_init(op)
    for step in range(1, 4):
        g = rng.normal(0, 1e-2, size=mlp.P)
        mlp.grads.copy_(torch.from_numpy(g.astype(np.float32)))
        mlp.adam(lr=1e-3)
        op = M.adam_step(op, [(g.astype(np.float32).astype(np.float64), np.zeros(1))], st, lr=1e-3)
        np.testing.assert_allclose(mlp.params.cpu().numpy(), op[0][0], rtol=1e-5, atol=1e-7)
    mlp.close()


def test_fused_step_equals_separate_calls_and_overfits(S, ctx):
    plain, sur = S
    a = sur.MLP(ctx, 32, 64, 16, max_batch=128, seed=7)
    b = sur.MLP(ctx, 32, 64, 16, max_batch=128, seed=7)
    x, t = batch(96, 32, 16, 8)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    first = None
    for it in range(300):
        la = a.train_step(xd, td, lr=3e-3)
        b.loss_raw(xd, td)
        b.backward_raw(b.params, None, 96, b.grads)
        b.adam(lr=3e-3)
        if it in (0, 1, 7):
            torch.cuda.synchronize()
            assert torch.equal(a.params, b.params), it
        if first is None:
            first = float(la.item())
    last = float(a.loss_raw(xd, td).item())
    assert last < 0.05 * first, (first, last)
    with pytest.raises(Exception):
        b.backward_raw(b.params, None, 95, b.grads)   # no kept forward of that batch
    a.close()
    b.close()
