"""GPU serving pieces: the judge (plain composed values of given subsets, and
the surrogate-disagreement flags), masked re-scoring, and the server's
fallback to the plain models."""
import numpy as np
import pytest
import torch

from synthgen import make_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_1910_07776_amd import plain as G
    ctx = G.Context(0)
    tr = make_batch(77, range(5000, 5256), 128, 12, brange=(0, 12))
    te = make_batch(77, range(300), 128, 12, brange=(0, 12))
    G.fit(ctx, G.Plan(ctx, tr.nopts, tr.opt_ids, 128, 12), torch.from_numpy(tr.counters).cuda(),
          torch.from_numpy(tr.cycles).cuda())
    p = G.Plan(ctx, te.nopts, te.opt_ids, 128, 12)
    c, cy = torch.from_numpy(te.counters).cuda(), torch.from_numpy(te.cycles).cuda()
    yield G, ctx, te, p, c, cy
    ctx.close()


def test_judge_is_bit_identical_to_the_fused_table(env):
    G, ctx, te, p, c, cy = env
    table, _ = G.predict(ctx, p, c, cy)
    rng = np.random.default_rng(3)
    C = 6
    cand = np.empty((te.K, C), np.int32)
    for k in range(te.K):
        cand[k] = rng.integers(0, 1 << te.nopts[k], size=C)
    cand[::7, 2] = -1
    out = G.judge(ctx, p, c, cy, torch.from_numpy(cand).cuda())
    G.sync(ctx)
    t, o = table.cpu().numpy(), out.cpu().numpy()
    for k in range(te.K):
        for j in range(C):
            S = cand[k, j]
            if S < 0:
                assert np.isnan(o[k, j])
            else:
                assert o[k, j] == t[te.row_off[k] + S], (k, S)   # bit-identical


def test_judge_flags_disagreements(env):
    G, ctx, te, p, c, cy = env
    table, _ = G.predict(ctx, p, c, cy)
    t = table.cpu().numpy()
    rng = np.random.default_rng(4)
    cand = np.full((te.K, 3), -1, np.int32)
    ref = np.zeros((te.K, 3), np.float32)
    want = np.zeros(te.K, np.int32)
    for k in range(te.K):
        if te.nopts[k] == 0:
            continue
        cand[k] = rng.integers(1, 1 << te.nopts[k], size=3)
        ref[k] = t[te.row_off[k] + cand[k]]
        j = rng.integers(0, 4)
        if j < 3:
            delta = rng.choice([0.05, -0.05, 0.2, -0.3])
            ref[k, j] += delta
            want[k] = abs(delta) > 0.1
    flag = torch.full((te.K,), 7, dtype=torch.int32, device="cuda")
    G.judge(ctx, p, c, cy, torch.from_numpy(cand).cuda(), ref=torch.from_numpy(ref).cuda(), tol=0.1, flag=flag)
    G.sync(ctx)
    assert np.array_equal(flag.cpu().numpy(), want)


def test_masked_rescoring(env):
    G, ctx, te, p, c, cy = env
    full = [x.clone() for x in G.suggest(ctx, p, c, cy)]
    rng = np.random.default_rng(5)
    mask = (rng.random(te.K) < 0.3).astype(np.int32)
    out = {"idx": torch.full((te.K, 3), -9, dtype=torch.int32, device="cuda"),
           "score": torch.full((te.K, 3), -9.0, device="cuda"),
           "count": torch.full((te.K,), -9, dtype=torch.int32, device="cuda"),
           "table": torch.full((te.N,), -9.0, device="cuda")}
    G.suggest_subset(ctx, p, c, cy, torch.from_numpy(mask).cuda(), out)
    G.sync(ctx)
    for k in range(te.K):
        r = slice(te.row_off[k], te.row_off[k + 1])
        if mask[k]:
            assert torch.equal(out["idx"][k], full[0][k]) and torch.equal(out["count"][k], full[2][k])
            assert torch.equal(out["table"][r], full[3][r])
        else:
            assert (out["idx"][k] == -9).all() and out["count"][k] == -9 and (out["table"][r] == -9).all()


def test_server_falls_back_to_plain_exactly(env):
    G, ctx, te, p, c, cy = env
    from paper_1910_07776_amd import serve, surrogate as Sg
    from synthgen.torch_world import TorchWorld
    tw = TorchWorld(77, 128, 12, B=6)
    cnt, cyc, _ = tw.chunk(3, 200)
    q = G.Plan(ctx, np.full(200, 6, np.int32), np.tile(np.arange(6, dtype=np.int32), 200), 128, 12)
    plain_out = G.suggest(ctx, q, cnt, cyc)
    bad = Sg.MLP(ctx, 128, 512, 64, max_batch=256, seed=9)
    bad.params.mul_(40.0)   # a broken surrogate: every kernel must be rejected
    srv = serve.Server(ctx, {6: bad}, n=3, tol=0.1)
    out = {"idx": torch.empty((200, 3), dtype=torch.int32, device="cuda"),
           "score": torch.empty((200, 3), device="cuda"),
           "count": torch.empty(200, dtype=torch.int32, device="cuda"), "table": None}
    flag = srv.answer(q, cnt, cyc, out)
    G.sync(ctx)
    assert int(flag.sum()) == 200
    assert torch.equal(out["idx"], plain_out[0]) and torch.equal(out["count"], plain_out[2])
    assert torch.equal(torch.nan_to_num(out["score"], nan=-7.0), torch.nan_to_num(plain_out[1], nan=-7.0))
    # a query size without a surrogate: plain path for all of it
    srv2 = serve.Server(ctx, {}, n=3)
    out2 = {k: torch.empty_like(v) if v is not None else None for k, v in out.items()}
    assert srv2.answer(q, cnt, cyc, out2) is None
    assert torch.equal(out2["idx"], plain_out[0])
    # the real-time loop on a few Poisson arrivals
    queries = [(q, cnt, cyc, out, serve.Server.footprint(200, 6, 128))] * 20
    st = serve.run_loop(srv, queries, serve.poisson_arrivals(20, 2000.0, 1))
    assert st["queries"] == 20 and st["p50_ms"] <= st["p99_ms"]
    bad.close()
