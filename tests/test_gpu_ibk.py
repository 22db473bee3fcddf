"""GPU instance-based Tier 2 model (IBK, k nearest neighbours) against the
FP64 oracle.  The GPU's neighbours are exact: its FP32 candidates are
re-ranked by FP64 distance and certified (or searched again in FP64), so
every neighbour set equals the oracle's and every prediction matches it to
1e-5 on the speedup scale (FP32 outputs) or 1e-9 (FP64 outputs); no query is
skipped.  The number of queries the library searched again is reported."""
import numpy as np
import pytest
import torch

from oracle import knn as N
from oracle import plain as P
from oracle.checks import check_list
from synthgen import make_batch

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("dtype,E,k", [(torch.float32, 128, 10), (torch.float64, 128, 10),
                                       (torch.float64, 40, 10), (torch.float32, 37, 3), (torch.float32, 96, 16),
                                       (torch.float32, 256, 10), (torch.float32, 200, 1)])
def test_ibk_matches_oracle(G, ctx, dtype, E, k):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    rtol = 1e-5 if dtype == torch.float32 else 1e-9
    tr = make_batch(31, range(4000, 4048), E, 6, brange=(2, 6), dtype=npdt)
    te = make_batch(31, range(40), E, 6, brange=(0, 6), dtype=npdt)
    ptr = G.Plan(ctx, tr.nopts, tr.opt_ids, E, 6, dtype=dtype)
    G.ibk_fit(ctx, ptr, dev(tr.counters), dev(tr.cycles), k=k)
    db = N.database(tr, 6)
    assert np.array_equal(G.ibk_counts(ctx, 6), [len(db["y"].get(o, [])) for o in range(6)])
    p = G.Plan(ctx, te.nopts, te.opt_ids, E, 6, dtype=dtype)
    c, cy = dev(te.counters), dev(te.cycles)
    table_g, grid = G.ibk_predict(ctx, p, c, cy, grid=True)
    n_grid = G.ibk_exact_count(ctx, p)
    table_e, _ = G.ibk_predict(ctx, p, c, cy)
    idx, score, count, table_s = G.ibk_suggest(ctx, p, c, cy)
    n_edges = G.ibk_exact_count(ctx, p)
    G.sync(ctx)
    print(f"E={E} k={k} {dtype}: queries searched again in FP64: grid {n_grid}, edges {n_edges}")
    # the chain-edge form and the grid form run the same searches
    assert torch.equal(table_g, table_e) and torch.equal(table_s, table_e)
    go = N.predict_grid(db, te, k, Bmax=p.Bmax)
    g = grid.cpu().numpy().astype(np.float64)
    pred = ~np.isnan(go)
    assert np.array_equal(~np.isnan(g), pred)
    ok = close(g[pred], go[pred], rtol)
    assert ok.all(), (np.flatnonzero(~ok)[:10], g[pred][~ok][:5], go[pred][~ok][:5])
    # every composed table and suggestion list
    to = P.compose(go, te)
    t = table_e.cpu().numpy().astype(np.float64)
    assert close(t, to, rtol).all()
    idx, score, count = idx.cpu().numpy(), score.cpu().numpy(), count.cpu().numpy()
    for kk in range(te.K):
        r0, r1 = int(te.row_off[kk]), int(te.row_off[kk + 1])
        errs = check_list(idx[kk, :count[kk]], score[kk, :count[kk]], to[r0:r1], P.TAU, 3, rtol, first=1)
        assert not errs, (kk, errs)


def test_one_neighbour_returns_the_training_labels(G, ctx):
    tr = make_batch(32, range(24), 128, 6, brange=(1, 6))
    p = G.Plan(ctx, tr.nopts, tr.opt_ids, 128, 6)
    c, cy = dev(tr.counters), dev(tr.cycles)
    G.ibk_fit(ctx, p, c, cy, k=1)
    _, grid = G.ibk_predict(ctx, p, c, cy, grid=True)
    G.sync(ctx)
    g = grid.cpu().numpy()
    opt, before, after, kern, S, b = P.candidate_pairs(tr.nopts, tr.opt_ids, tr.opt_off, tr.row_off)
    y = P.pair_labels(tr.cycles, before, after)
    np.testing.assert_allclose(g[before, b], y.astype(np.float32), rtol=1e-6, atol=1e-7)


def test_ibk_full_size(G, ctx):
    """512 training and 512 test kernels of 64 versions x 128 events (16,384
    samples per optimisation, 32,256 chain-edge searches) in the launch the
    benchmark times: 1,000 sampled chain edges against the oracle's search,
    every one compared."""
    tr = make_batch(1910, range(10 ** 6, 10 ** 6 + 512), 128, 6)
    te = make_batch(1910, range(512), 128, 6)
    ptr = G.Plan(ctx, tr.nopts, tr.opt_ids, 128, 6)
    G.ibk_fit(ctx, ptr, dev(tr.counters), dev(tr.cycles), k=10)
    p = G.Plan(ctx, te.nopts, te.opt_ids, 128, 6)
    idx, score, count, table = G.ibk_suggest(ctx, p, dev(te.counters), dev(te.cycles))
    n_exact = G.ibk_exact_count(ctx, p)
    G.sync(ctx)
    print(f"queries searched again in FP64: {n_exact} of {te.N - te.K}")
    assert n_exact < 0.05 * (te.N - te.K)
    t = table.cpu().numpy().astype(np.float64)
    db = N.database(tr, 6)
    z = P.standardize(P.features(te.counters, te.cycles), db["mu"], db["sigma"])
    rng = np.random.default_rng(5)
    for r in rng.choice(np.flatnonzero(np.arange(te.N) % 64 != 0), size=1000, replace=False):
        S = int(r % 64)
        b = S.bit_length() - 1                      # the last step of S's chain
        want = N.predict_one(db, z[r - (1 << b)], b, 10)
        got = t[r] - t[r - (1 << b)]                 # the edge, from the composed table
        assert abs(got - want) <= 2e-5 * (1 + abs(want)) + 4e-6 * abs(t[r]), (r, got, want)


def test_ibk_errors(G, ctx):
    from paper_1910_07776_amd._abi import SuggError
    tr = make_batch(33, range(8), 128, 6, brange=(3, 3))
    ids = np.tile(np.arange(3, dtype=np.int32), 8)       # samples of ids 0..2 only
    p = G.Plan(ctx, tr.nopts, ids, 128, 6)
    c, cy = dev(tr.counters), dev(tr.cycles)
    for k in (0, 17):
        with pytest.raises(SuggError) as e:
            G.ibk_fit(ctx, p, c, cy, k=k)
        assert e.value.name == "SUGG_E_ARG"
    G.ibk_fit(ctx, p, c, cy)
    assert np.array_equal(G.ibk_counts(ctx, 6), [32, 32, 32, 0, 0, 0])
    one = make_batch(33, range(100, 101), 128, 6, brange=(1, 1))
    q = G.Plan(ctx, np.array([1], np.int32), np.array([4], np.int32), 128, 6)
    with pytest.raises(SuggError) as e:
        G.ibk_predict(ctx, q, dev(one.counters), dev(one.cycles))
    assert e.value.name == "SUGG_E_UNTRAINED_OPT"
    ctx2 = G.Context(0)
    with pytest.raises(SuggError) as e:
        G.ibk_predict(ctx2, G.Plan(ctx2, np.array([1], np.int32), np.array([0], np.int32), 128, 6),
                      dev(one.counters), dev(one.cycles))
    assert e.value.name == "SUGG_E_STATE"
    ctx2.close()


def test_ibk_bad_counters_give_nan_and_the_status(G, ctx):
    """A non-positive counter makes its row's feature vector NaN: the device
    status reports it, that row's searches find no neighbour and predict NaN,
    and every other prediction stays finite."""
    from paper_1910_07776_amd._abi import SuggError
    tr = make_batch(34, range(16), 128, 6, brange=(4, 4))
    ids4 = np.tile(np.arange(4, dtype=np.int32), 16)
    G.ibk_fit(ctx, G.Plan(ctx, tr.nopts, ids4, 128, 6), dev(tr.counters), dev(tr.cycles), k=10)
    G.sync(ctx)
    te = make_batch(34, range(100, 104), 128, 6, brange=(2, 2))
    p = G.Plan(ctx, np.full(4, 2, np.int32), np.tile(np.arange(2, dtype=np.int32), 4), 128, 6)
    c = te.counters.copy()
    c[5, 3] = -1.0                                        # kernel 1, version 1
    table, grid = G.ibk_predict(ctx, p, dev(c), dev(te.cycles), grid=True)
    with pytest.raises(SuggError) as e:
        G.sync(ctx)
    assert e.value.name == "SUGG_E_BAD_COUNTER"
    g = grid.cpu().numpy()
    assert np.isnan(g[5]).all()                           # bit 1 of version 1: no neighbour
    others = np.ones(16, dtype=bool)
    others[5] = False
    want = np.zeros((16, 2), dtype=bool)
    for r in range(16):
        S = r % 4
        want[r] = [(S >> b) & 1 == 0 for b in range(2)]
    assert np.isfinite(g[others][want[others]]).all()
