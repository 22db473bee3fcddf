"""GPU model-tree Tier 2 model (M5P) against the FP64 oracle.

The trees are induced on the host from FP64 features computed on the GPU, so
they must equal the oracle's node for node (tested feature, children, case
counts; thresholds to rounding).  A prediction is formed in FP64 whatever the
plan's dtype (features from the counters, the walk's tests, the leaf model),
so every walk takes the oracle's branch: no prediction is skipped (a test
feature within 1e-12 of a threshold on its path, where FP64 rounding alone
could decide, is asserted absent), and every prediction, composed entry and
suggestion list matches the oracle to 1e-5 on the speedup scale for FP32
outputs and 1e-9 for FP64 ones."""
import numpy as np
import pytest
import torch

from oracle import m5p as M
from oracle import plain as P
from oracle.checks import check_list
from synthgen import make_batch

pytestmark = pytest.mark.gpu

MARGIN = 1e-12
RTOL = {torch.float32: 1e-5, torch.float64: 1e-9}


@pytest.fixture(scope="module")
def G():
    from paper_1910_07776_amd import plain
    return plain


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def close(got, want, rtol):
    return np.abs(np.exp(got) - np.exp(want)) <= rtol * np.exp(want)


def assert_same_tree(got, want):
    assert np.array_equal(got["feat"], want["feat"])
    assert np.array_equal(got["left"], want["left"]) and np.array_equal(got["right"], want["right"])
    assert np.array_equal(got["count"], want["n"])
    inner = want["feat"] >= 0
    assert np.isnan(got["thr"][~inner]).all()
    np.testing.assert_allclose(got["thr"][inner], want["thr"][inner], rtol=0, atol=1e-11)


@pytest.mark.parametrize("dtype,E,min_leaf,smooth_k", [(torch.float32, 128, 4, 15.0), (torch.float64, 128, 4, 15.0),
                                                       (torch.float32, 37, 4, 15.0), (torch.float64, 40, 2, 0.0),
                                                       (torch.float32, 200, 6, 5.0), (torch.float32, 1, 4, 15.0),
                                                       (torch.float64, 16, 100000, 15.0)])
def test_m5p_matches_oracle(G, ctx, dtype, E, min_leaf, smooth_k):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    tr = make_batch(41, range(5000, 5048), E, 6, brange=(2, 6), dtype=npdt)
    te = make_batch(41, range(40), E, 6, brange=(0, 6), dtype=npdt)
    ptr = G.Plan(ctx, tr.nopts, tr.opt_ids, E, 6, dtype=dtype)
    G.m5p_fit(ctx, ptr, dev(tr.counters), dev(tr.cycles), min_leaf=min_leaf, smooth_k=smooth_k)
    model = M.fit(tr, 6, min_leaf=min_leaf, smooth_k=smooth_k)
    for o, want in model["trees"].items():
        assert_same_tree(G.m5p_tree(ctx, o), want)
    p = G.Plan(ctx, te.nopts, te.opt_ids, E, 6, dtype=dtype)
    c, cy = dev(te.counters), dev(te.cycles)
    table_g, grid = G.m5p_predict(ctx, p, c, cy, grid=True)
    table_e, _ = G.m5p_predict(ctx, p, c, cy)
    idx, score, count, table_s = G.m5p_suggest(ctx, p, c, cy)
    G.sync(ctx)
    # the grid form and the chain-edge form evaluate the same walks
    assert torch.equal(table_g, table_e) and torch.equal(table_s, table_e)
    go, margin = M.predict_grid(model, te, Bmax=p.Bmax)
    g = grid.cpu().numpy().astype(np.float64)
    pred = ~np.isnan(go)
    assert np.array_equal(~np.isnan(g), pred)
    assert (margin[pred] > MARGIN).all()
    ok = close(g[pred], go[pred], RTOL[dtype])
    print(f"{dtype} E={E}: {pred.sum()} predictions, largest difference "
          f"{np.max(np.abs(g[pred] - go[pred])) if pred.any() else 0:.2e}")
    assert ok.all(), (np.flatnonzero(~ok)[:10], np.max(np.abs(g[pred] - go[pred])))
    to = P.compose(go, te)
    t = table_e.cpu().numpy().astype(np.float64)
    assert close(t, to, RTOL[dtype]).all()
    idx, score, count = idx.cpu().numpy(), score.cpu().numpy(), count.cpu().numpy()
    for kk in range(te.K):
        r0, r1 = int(te.row_off[kk]), int(te.row_off[kk + 1])
        errs = check_list(idx[kk, :count[kk]], score[kk, :count[kk]], to[r0:r1], P.TAU, 3, RTOL[dtype], first=1)
        assert not errs, (kk, errs)


def test_m5p_kernels_above_64_versions(G, ctx):
    """Plans with kernels of up to 256 versions take the tiled path with a
    separate composition; tables and lists as in the oracle."""
    tr = make_batch(45, range(6000, 6024), 64, 8, brange=(3, 8))
    te = make_batch(45, range(12), 64, 8, brange=(5, 8))
    G.m5p_fit(ctx, G.Plan(ctx, tr.nopts, tr.opt_ids, 64, 8), dev(tr.counters), dev(tr.cycles))
    model = M.fit(tr, 8)
    p = G.Plan(ctx, te.nopts, te.opt_ids, 64, 8)
    assert p.Bmax > 6
    idx, score, count, table = G.m5p_suggest(ctx, p, dev(te.counters), dev(te.cycles))
    G.sync(ctx)
    go, margin = M.predict_grid(model, te, Bmax=p.Bmax)
    assert (margin[~np.isnan(go)] > MARGIN).all()
    to = P.compose(go, te)
    t = table.cpu().numpy().astype(np.float64)
    assert close(t, to, RTOL[torch.float32]).all()
    idx, score, count = idx.cpu().numpy(), score.cpu().numpy(), count.cpu().numpy()
    for kk in range(te.K):
        r0, r1 = int(te.row_off[kk]), int(te.row_off[kk + 1])
        assert not check_list(idx[kk, :count[kk]], score[kk, :count[kk]], to[r0:r1], P.TAU, 3,
                              RTOL[torch.float32], first=1)


def test_m5p_full_size(G, ctx):
    """512 training kernels of 64 versions x 128 FP32 events (16,384 pairs per
    optimisation): the trees of two optimisations node for node, and every
    one of the 512 test kernels' predictions of those two optimisations
    (16,384 each) against the oracle's walks."""
    tr = make_batch(1910, range(10 ** 6, 10 ** 6 + 512), 128, 6)
    te = make_batch(1910, range(512), 128, 6)
    ptr = G.Plan(ctx, tr.nopts, tr.opt_ids, 128, 6)
    G.m5p_fit(ctx, ptr, dev(tr.counters), dev(tr.cycles))
    p = G.Plan(ctx, te.nopts, te.opt_ids, 128, 6)
    _, grid = G.m5p_predict(ctx, p, dev(te.counters), dev(te.cycles), grid=True)
    G.sync(ctx)
    g = grid.cpu().numpy().astype(np.float64)
    x = P.features(tr.counters, tr.cycles)
    mu, sigma = P.column_stats(x)
    z = P.standardize(x, mu, sigma)
    opt, before, after, *_ = P.candidate_pairs(tr.nopts, tr.opt_ids, tr.opt_off, tr.row_off)
    y = P.pair_labels(tr.cycles, before, after)
    zt = P.standardize(P.features(te.counters, te.cycles), mu, sigma)
    for o in (0, 5):
        sel = np.flatnonzero(opt == o)
        tree = M.build(z[before[sel]], y[sel])
        assert_same_tree(G.m5p_tree(ctx, o), tree)
        rows = [r for r in range(te.N) if not ((r % 64) >> o) & 1]
        for r in rows:
            want, margin = M.predict_one(tree, zt[r])
            assert margin > MARGIN, (o, r, margin)
            assert close(g[r, o], want, RTOL[torch.float32]), (o, r, g[r, o], want)
        print(f"optimisation {o}: {len(rows)} predictions match the oracle")


def test_m5p_errors(G, ctx):
    from paper_1910_07776_amd._abi import SuggError
    tr = make_batch(43, range(8), 128, 6, brange=(3, 3))
    ids = np.tile(np.arange(3, dtype=np.int32), 8)       # pairs of ids 0..2 only
    p = G.Plan(ctx, tr.nopts, ids, 128, 6)
    c, cy = dev(tr.counters), dev(tr.cycles)
    for kw in ({"min_leaf": 0}, {"smooth_k": -1.0}, {"smooth_k": float("nan")}):
        with pytest.raises(SuggError) as e:
            G.m5p_fit(ctx, p, c, cy, **kw)
        assert e.value.name == "SUGG_E_ARG"
    bad = tr.counters.copy()
    bad[3, 7] = 0.0
    with pytest.raises(SuggError) as e:
        G.m5p_fit(ctx, p, dev(bad), cy)
    assert e.value.name == "SUGG_E_BAD_COUNTER"
    with pytest.raises(SuggError):
        G.sync(ctx)                                       # the status word saw it too
    G.m5p_fit(ctx, p, c, cy)
    for o in range(3):
        assert G.m5p_tree(ctx, o)["count"][0] == 32
    with pytest.raises(SuggError) as e:
        G.m5p_tree(ctx, 4)
    assert e.value.name == "SUGG_E_UNTRAINED_OPT"
    one = make_batch(43, range(100, 101), 128, 6, brange=(1, 1))
    q = G.Plan(ctx, np.array([1], np.int32), np.array([4], np.int32), 128, 6)
    with pytest.raises(SuggError) as e:
        G.m5p_predict(ctx, q, dev(one.counters), dev(one.cycles))
    assert e.value.name == "SUGG_E_UNTRAINED_OPT"
    q64 = G.Plan(ctx, np.array([1], np.int32), np.array([0], np.int32), 64, 6)
    with pytest.raises(SuggError) as e:
        G.m5p_predict(ctx, q64, dev(np.ones((2, 64), np.float32)), dev(np.ones(2, np.float32)))
    assert e.value.name == "SUGG_E_SHAPE"
    ctx2 = G.Context(0)
    with pytest.raises(SuggError) as e:
        G.m5p_predict(ctx2, G.Plan(ctx2, np.array([1], np.int32), np.array([0], np.int32), 128, 6),
                      dev(one.counters), dev(one.cycles))
    assert e.value.name == "SUGG_E_STATE"
    ctx2.close()


def test_m5p_bad_counter_sets_the_status(G, ctx):
    tr = make_batch(44, range(16), 128, 6, brange=(4, 4))
    ids4 = np.tile(np.arange(4, dtype=np.int32), 16)
    G.m5p_fit(ctx, G.Plan(ctx, tr.nopts, ids4, 128, 6), dev(tr.counters), dev(tr.cycles))
    G.sync(ctx)
    from paper_1910_07776_amd._abi import SuggError
    te = make_batch(44, range(100, 104), 128, 6, brange=(2, 2))
    p = G.Plan(ctx, np.full(4, 2, np.int32), np.tile(np.arange(2, dtype=np.int32), 4), 128, 6)
    c = te.counters.copy()
    c[5, 3] = -1.0
    table, _ = G.m5p_predict(ctx, p, dev(c), dev(te.cycles))
    with pytest.raises(SuggError) as e:
        G.sync(ctx)
    assert e.value.name == "SUGG_E_BAD_COUNTER"
    G.sync(ctx)                                           # reported once
    t = table.cpu().numpy()
    assert np.isfinite(t[[0, 1, 2, 3, 8, 9, 10, 11, 12, 13, 14, 15]]).all()
