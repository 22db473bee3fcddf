"""GPU surrogate MLP (BF16 matrix cores, hand-written backward, Adam) against
the FP64 oracle evaluated at the same BF16 rounding points (weights, input and
hidden activations rounded to bfloat16).  Tolerance 3e-2 relative for BF16
results, element by element, relative to max(|reference|, floor) with the
floor the tensor's root-mean-square reference value (an element of a sum of
thousands of signed terms can be near zero, where a relative error says
nothing); FP32 Adam 1e-5.  The batch sizes the benchmark runs (4096 for
training, 65,536 for inference) are compared too, with the launched
matrix-core instances reported by the library."""
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
    """max over elements of |a - b| / max(|b|, rms(b))."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    floor = max(float(np.sqrt(np.mean(b * b))), 1e-30)
    return float((np.abs(a - b) / np.maximum(np.abs(b), floor)).max())


def launch_info(mlp):
    import ctypes as C
    from paper_1910_07776_amd import _abi as A
    info = np.zeros(32, np.int32)
    assert A.lib().sugg_mlp_launch_info(mlp.h, info.ctypes.data_as(A._PI32)) == 0
    return info.reshape(8, 4)


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
    # through torch.autograd (the output gradient comes from torch's MSE):
    # the same oracle gradients
    p = mlp.params.clone().requires_grad_(True)
    yy = sur.SurrogateFn.apply(xd, p, mlp)
    ((yy - td) ** 2).mean().backward()
    torch.cuda.synchronize()
    ga = mlp.unflatten(p.grad.cpu().numpy().astype(np.float64))
    for li, (Wn, bn) in enumerate((("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
        assert rel(ga[Wn], go[li][0].T) < BF16_RTOL, Wn
        assert rel(ga[bn], go[li][1]) < BF16_RTOL, bn
    mlp.close()


@pytest.mark.parametrize("B", [4096, 65536])
def test_forward_at_benchmark_batches(S, ctx, B):
    """Inference forward at the batches the benchmark times (65,536 kernels
    in one call for the surrogate-vs-plain comparison; 4096 in training),
    every output element against the oracle."""
    plain, sur = S
    mlp = sur.MLP(ctx, 128, 512, 64, max_batch=B, seed=21)
    x, _ = batch(B, 128, 64, 22)
    y = mlp(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    info = launch_info(mlp)
    print(f"batch {B}: forward instances (tile rows, tile cols, splits, K stage) {info[:3].tolist()}")
    yo, _ = M.forward_bf16(oracle_params(mlp, mlp.params.cpu().numpy()), x)
    err = rel(y.cpu().numpy(), yo)
    print(f"batch {B}: max element error {err:.2e}")
    assert err < BF16_RTOL
    # every layer ran instances without bounds checks: 64 x 64 tiles with
    # K stages of 128 at 4096 kernels, 128 x 128 tiles with K stages of 32
    # for the hidden layers at 65,536
    assert info[0, 3] > 0 and info[1, 3] > 0 and info[2, 3] > 0
    if B == 65536:
        assert info[0].tolist() == [128, 128, 1, 32] and info[1].tolist() == [128, 128, 1, 32]
    else:
        assert info[0].tolist() == [64, 64, 1, 128] and info[1].tolist() == [64, 64, 1, 128]
    mlp.close()


def test_training_gradients_at_batch_4096(S, ctx):
    """Loss and hand-written backward at the training batch (4096): the
    weight gradients run split over the batch; every gradient element
    against the oracle's backward of the same BF16-rounded forward."""
    plain, sur = S
    B = 4096
    mlp = sur.MLP(ctx, 128, 512, 64, max_batch=B, seed=23)
    x, t = batch(B, 128, 64, 24)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss = mlp.loss_raw(xd, td)
    g = mlp.backward_raw(mlp.params, None, B, torch.empty_like(mlp.params))
    torch.cuda.synchronize()
    info = launch_info(mlp)
    print(f"backward instances (tile rows, tile cols, splits, K stage) {info[3:].tolist()}")
    assert all(info[i, 2] > 1 for i in (3, 5, 7))   # the weight gradients were split over the batch
    op = oracle_params(mlp, mlp.params.cpu().numpy())
    pr = [(M.bf16_round(W), b) for W, b in op]
    y, cache = M.forward(pr, M.bf16_round(x), round_hidden=M.bf16_round)
    lo, dy = M.mse(y, t)
    assert abs(float(loss.item()) - lo) <= BF16_RTOL * lo
    go = M.backward(pr, cache, dy)
    gu = mlp.unflatten(g.cpu().numpy().astype(np.float64))
    for li, (Wn, bn) in enumerate((("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
        e_w, e_b = rel(gu[Wn], go[li][0].T), rel(gu[bn], go[li][1])
        print(f"{Wn} {e_w:.2e} {bn} {e_b:.2e}")
        assert e_w < BF16_RTOL, Wn
        assert e_b < BF16_RTOL, bn
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


@pytest.mark.parametrize("dims,n,batch", [((128, 512, 64), 20000, 4096), ((32, 64, 16), 700, 96)])
def test_epoch_call_equals_steps_on_gathered_batches(S, ctx, dims, n, batch):
    """sugg_mlp_train_epoch (gather in the first kernel, targets by row
    index, bias gradients with the split-K sums, Adam writing the BF16
    weights) against train_step on index_select'ed batches: parameters, Adam
    moments and every loss bit-identical."""
    plain, sur = S
    i, h, o = dims
    rng = np.random.default_rng(12)
    X = torch.tensor(rng.normal(size=(n, i)), dtype=torch.float32, device="cuda")
    Y = torch.tensor(rng.normal(size=(n, o)) * 0.2, dtype=torch.float32, device="cuda")
    steps = 3
    perm = torch.tensor(rng.permutation(n)[:steps * batch], dtype=torch.int32, device="cuda")
    a = sur.MLP(ctx, i, h, o, max_batch=batch, seed=4)
    b = sur.MLP(ctx, i, h, o, max_batch=batch, seed=4)
    la = a.train_epoch(X, Y, perm, batch, lr=2e-3)
    lb = []
    for s in range(steps):
        idx = perm[s * batch:(s + 1) * batch].long()
        lb.append(b.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr=2e-3).clone())
    plain.sync(ctx)
    assert torch.equal(a.params, b.params) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
    assert torch.equal(la, torch.cat(lb)) and a.step == b.step == steps
    # an index outside the training set reads row 0 and is reported, nothing faults
    bad = perm.clone()
    bad[5] = n + 3
    a.train_epoch(X, Y, bad, batch, lr=2e-3)
    with pytest.raises(Exception):
        plain.sync(ctx)
    plain.sync(ctx)   # the error was reported once
    a.close()
    b.close()


@pytest.mark.parametrize("out,n,tau", [(64, 3, 0.02), (128, 8, 0.0), (256, 3, 0.02), (64, 5, 0.3)])
def test_infer_rank_equals_infer_then_rank(S, ctx, out, n, tau):
    """Frozen inference with Tier 3 in the output layer's epilogue (outputs
    of 64 or 128 columns; the row ranking kernel for wider ones) against
    inference followed by sugg_rank_suggest: same outputs, same lists, on a
    batch that is not a whole number of tiles."""
    plain, sur = S
    B = 4999
    mlp = sur.MLP(ctx, 128, 512, out, max_batch=B, seed=31)
    rng = np.random.default_rng(32)
    x = torch.tensor(rng.normal(size=(B, 128)), dtype=torch.float32, device="cuda")
    mlp.freeze()
    y = mlp.infer(x)
    y_fwd = mlp(x)                      # the same parameters through forward
    y2 = torch.empty_like(y)
    idx, sc, cnt = mlp.infer_rank(x, n=n, tau=tau, skip=1, y=y2)
    idx0, sc0, cnt0 = mlp.infer_rank(x, n=n, tau=tau, skip=1)   # without the outputs
    seg = torch.arange(0, B + 1, dtype=torch.int64, device="cuda") * out
    ri, rs, rc = plain.rank_suggest(ctx, y.view(-1), seg, n=n, tau=tau, skip_head=1)
    plain.sync(ctx)
    assert torch.equal(y, y2) and torch.equal(y, y_fwd)
    for a, b, c in ((idx, sc, cnt), (idx0, sc0, cnt0)):
        assert torch.equal(a, ri) and torch.equal(c, rc)
        assert torch.equal(torch.nan_to_num(b, nan=-7.0), torch.nan_to_num(rs, nan=-7.0))
    if tau >= 0.3:
        assert int(rc.min()) < n   # short lists where tau bites
    info = launch_info(mlp)
    if out <= 128:   # the ranking epilogue: one tile row holds a whole output row
        assert info[2, 0] == 128 and info[2, 1] == out
    mlp.close()


def test_surrogate_suggest_in_one_call(S, ctx):
    """sugg_surrogate_suggest (baseline features written in BF16 into the
    network's input, the network, Tier 3 in its output layer) against
    load_features (baseline rows) + infer_rank and infer: identical lists
    and table."""
    plain, sur = S
    from synthgen import make_batch
    from synthgen.torch_world import TorchWorld
    tr = make_batch(41, range(9000, 9128), 128, 6)
    plain.fit(ctx, plain.Plan(ctx, tr.nopts, tr.opt_ids, 128, 6), torch.from_numpy(tr.counters).cuda(),
              torch.from_numpy(tr.cycles).cuda())
    tw = TorchWorld(41, 128, 6)
    K = 3001
    c, cy, _ = tw.chunk(2, K)
    p = plain.Plan(ctx, np.full(K, 6, np.int32), np.tile(np.arange(6, dtype=np.int32), K), 128, 6)
    mlp = sur.MLP(ctx, 128, 512, 64, max_batch=K, seed=33).freeze()
    idx, sc, cnt, table = plain.surrogate_suggest(ctx, p, mlp, c, cy, table=True)
    zz = plain.load_features(ctx, p, c, cy, baseline=True)
    ri, rs, rc = mlp.infer_rank(zz, n=3, tau=plain.TAU, skip=1)
    y = mlp.infer(zz)
    plain.sync(ctx)
    assert torch.equal(idx, ri) and torch.equal(cnt, rc)
    assert torch.equal(torch.nan_to_num(sc, nan=-7.0), torch.nan_to_num(rs, nan=-7.0))
    assert torch.equal(table, y)
    mlp.close()


def test_trained_surrogate_gains_over_baseline_only_method(S, ctx):
    """What the trained network gains over the method without it: from the
    same input (a kernel's baseline profile only), the surrogate's speedup
    MAPE against the generator's truth beats the sum of the plain models'
    single-optimisation predictions for the baseline version.  The plain
    composed table, which needs all 64 profiled versions, is reported."""
    plain, sur = S
    from synthgen import make_batch
    from synthgen.torch_world import TorchWorld
    tr = make_batch(1910, range(10 ** 6, 10 ** 6 + 2048), 128, 6)
    p = plain.Plan(ctx, tr.nopts, tr.opt_ids, 128, 6)
    plain.fit(ctx, p, torch.from_numpy(tr.counters).cuda(), torch.from_numpy(tr.cycles).cuda())
    tw = TorchWorld(1910, 128, 6)
    data = sur.build_dataset(ctx, tw, 131072, chunk=65536, chunk_base=0)
    val = sur.build_dataset(ctx, tw, 16384, chunk=16384, chunk_base=5000, with_truth=True, with_baseline_grid=True)
    plain.sync(ctx)
    mlp = sur.MLP(ctx, 128, 512, 64, max_batch=4096, seed=1)
    hist = sur.train(mlp, data["X"], data["Y"], epochs=12, lr=1e-3, val=(val["X"], val["T"]), check_every=12)
    m_sur = hist[-1]["val_mape"]
    # the method without the surrogate, from the same input: the sum over the
    # subset's optimisations of the plain models' baseline predictions
    S = torch.arange(64, device=val["G0"].device)
    bits = ((S[:, None] >> torch.arange(6, device=S.device)) & 1).float()
    m_add = sur.mape(val["G0"] @ bits.T, val["T"])
    m_plain = sur.mape(val["Y"], val["T"])
    print(f"MAPE surrogate {m_sur:.4f}  additive-from-baseline {m_add:.4f}  plain chain {m_plain:.4f}")
    assert hist[-1]["loss"] < hist[0]["loss"]
    assert m_sur < m_add
    mlp.close()
