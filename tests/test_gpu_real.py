"""The GPU path on real MI355X profiles (counters of 64 versions of two
programs measured with rocprofv3, paper_1910_07776_amd/profiling) against the
FP64 oracle on the same inputs: ridge tables, grids and suggestions, IBK
neighbours (exact) with their predictions, and M5P trees node for node with
their predictions (formed in FP64 on the GPU: 1e-5 on the speedup scale).

Tolerance of the FP32 ridge path on these data: real counters are strongly
correlated, so the ridge weights are large and cancel, and the FP32 rounding
of the features is amplified.  Each feature ln(c / cyc) comes from two FP32
base-2 logarithms (relative rounding 2^-24 each) and is standardised by the
column's sigma, so |dz_j| <= 2^-24 ln 2 (|log2 c_j| + |log2 cyc|) / sigma_j;
a prediction's error is then at most sum_j |w_j| |dz_j| plus the rounding of
its E-term dot product (E 2^-24 sum_j |w_j z_j|).  A composed entry may
differ by the sum of these bounds along its chain (plus 1e-6)."""
import numpy as np
import pytest
import torch

from oracle import knn as N
from oracle import m5p as M
from oracle import plain as P
from oracle.checks import check_list
from paper_1910_07776_amd.profiling import dataset as R

pytestmark = pytest.mark.gpu

EXPERIMENTS = {
    "one run -> all runs": (R.sweeps(0, runs=(0,)), R.sweeps(0)),
    "n-body -> gather": (R.sweeps(0), R.sweeps(1)),
    "inputs 0,1 -> input 2": (R.sweeps(None, inputs=(0, 1)), R.sweeps(None, inputs=(2,))),
}


@pytest.fixture(scope="module")
def G():
    from paper_1910_07776_amd import plain
    return plain


@pytest.fixture(scope="module")
def data():
    return R.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def chain_bounds(model, batch):
    """Per grid entry and per composed entry: the first-order bound above."""
    c = batch.counters.astype(np.float64)
    cyc = batch.cycles.astype(np.float64)
    z = P.standardize(P.features(c, cyc), model["mu"], model["sigma"])
    eps = 2.0 ** -24
    dz = eps * np.log(2) * (np.abs(np.log2(c)) + np.abs(np.log2(cyc))[:, None]) / model["sigma"]
    W = model["W"][:, :-1]
    edge = np.zeros((batch.N, 6))
    for k in range(batch.K):
        r0 = int(batch.row_off[k])
        for b in range(6):
            w = W[int(batch.opt_ids[6 * k + b])]
            rows = slice(r0, r0 + 64)
            edge[rows, b] = dz[rows] @ np.abs(w) + batch.E * eps * (np.abs(z[rows] * w)).sum(1)
    table = np.zeros(batch.N)
    for k in range(batch.K):
        r0 = int(batch.row_off[k])
        for S in range(1, 64):
            top = S.bit_length() - 1
            table[r0 + S] = table[r0 + S - (1 << top)] + edge[r0 + S - (1 << top), top]
    return edge + 1e-6, table + 1e-6


@pytest.mark.parametrize("name", list(EXPERIMENTS))
def test_ridge_on_real_profiles(G, data, name):
    tr_s, te_s = EXPERIMENTS[name]
    tr, te = R.batch(data, tr_s), R.batch(data, te_s)
    om = P.fit(tr, 6)
    ogrid, otab, _ = P.run(om, te)
    ctx = G.Context(0)
    try:
        G.fit(ctx, G.Plan(ctx, tr.nopts, tr.opt_ids, tr.E, 6), dev(tr.counters), dev(tr.cycles))
        p = G.Plan(ctx, te.nopts, te.opt_ids, te.E, 6)
        c, cy = dev(te.counters), dev(te.cycles)
        idx, score, count, table = G.suggest(ctx, p, c, cy)
        _, grid = G.predict(ctx, p, c, cy, grid=True)
        G.sync(ctx)
        eb, tb = chain_bounds(om, te)
        t = table.cpu().numpy().astype(np.float64)
        assert (np.abs(t - otab) <= tb).all(), np.max(np.abs(t - otab) / tb)
        g = grid.cpu().numpy().astype(np.float64)
        m = ~np.isnan(ogrid)
        assert np.array_equal(~np.isnan(g), m) and (np.abs(g[m] - ogrid[m]) <= eb[m]).all()
        idx, score, count = idx.cpu().numpy(), score.cpu().numpy(), count.cpu().numpy()
        for k in range(te.K):
            r0, r1 = te.row_off[k], te.row_off[k + 1]
            tol = float(np.max(tb[r0:r1]))
            assert not check_list(idx[k, :count[k]], score[k, :count[k]], otab[r0:r1], P.TAU, 3, tol, first=1), k
    finally:
        ctx.close()


@pytest.mark.parametrize("name", list(EXPERIMENTS))
def test_ibk_on_real_profiles(G, data, name):
    """IBK (k = 10) trained on some real profiles, predicting others: every
    grid prediction, composed entry and suggestion list against the oracle
    (the GPU's neighbours are exact, so the FP32 outputs match to 1e-5 on
    the speedup scale; no bound from the data is needed)."""
    tr_s, te_s = EXPERIMENTS[name]
    tr, te = R.batch(data, tr_s), R.batch(data, te_s)
    db = N.database(tr, 6)
    go = N.predict_grid(db, te, 10, Bmax=6)
    to = P.compose(go, te)
    ctx = G.Context(0)
    try:
        G.ibk_fit(ctx, G.Plan(ctx, tr.nopts, tr.opt_ids, tr.E, 6), dev(tr.counters), dev(tr.cycles), k=10)
        p = G.Plan(ctx, te.nopts, te.opt_ids, te.E, 6)
        c, cy = dev(te.counters), dev(te.cycles)
        _, grid = G.ibk_predict(ctx, p, c, cy, grid=True)
        idx, score, count, table = G.ibk_suggest(ctx, p, c, cy)
        n_exact = G.ibk_exact_count(ctx, p)
        G.sync(ctx)
        print(f"{name}: {n_exact} queries searched again in FP64")
        g = grid.cpu().numpy().astype(np.float64)
        m = ~np.isnan(go)
        assert np.array_equal(~np.isnan(g), m)
        assert (np.abs(np.exp(g[m]) - np.exp(go[m])) <= 1e-5 * np.exp(go[m])).all()
        t = table.cpu().numpy().astype(np.float64)
        assert (np.abs(np.exp(t) - np.exp(to)) <= 1e-5 * np.exp(to)).all()
        idx, score, count = idx.cpu().numpy(), score.cpu().numpy(), count.cpu().numpy()
        for k in range(te.K):
            r0, r1 = te.row_off[k], te.row_off[k + 1]
            assert not check_list(idx[k, :count[k]], score[k, :count[k]], to[r0:r1], P.TAU, 3, 1e-5, first=1), k
    finally:
        ctx.close()


def test_m5p_on_real_profiles(G, data):
    """Trees grown on the n-body program node for node, and their predictions
    for the gather program's versions (extrapolation: the node models' unique
    solutions matter when counters are collinear, as real ones are)."""
    tr, te = R.batch(data, R.sweeps(0)), R.batch(data, R.sweeps(1))
    model = M.fit(tr, 6)
    ctx = G.Context(0)
    try:
        G.m5p_fit(ctx, G.Plan(ctx, tr.nopts, tr.opt_ids, tr.E, 6), dev(tr.counters), dev(tr.cycles))
        for o, want in model["trees"].items():
            got = G.m5p_tree(ctx, o)
            assert np.array_equal(got["feat"], want["feat"]) and np.array_equal(got["count"], want["n"])
            assert np.array_equal(got["left"], want["left"]) and np.array_equal(got["right"], want["right"])
            inner = want["feat"] >= 0
            np.testing.assert_allclose(got["thr"][inner], want["thr"][inner], rtol=0, atol=1e-11)
        p = G.Plan(ctx, te.nopts, te.opt_ids, te.E, 6)
        _, grid = G.m5p_predict(ctx, p, dev(te.counters), dev(te.cycles), grid=True)
        G.sync(ctx)
        go, margin = M.predict_grid(model, te, Bmax=6)
        g = grid.cpu().numpy().astype(np.float64)
        m = ~np.isnan(go)
        assert np.array_equal(~np.isnan(g), m)
        # the GPU walks and evaluates in FP64 like the oracle: every prediction
        # compared (no test feature lies within FP64 rounding of a threshold)
        assert (margin[m] > 1e-12).all()
        assert (np.abs(np.exp(g[m]) - np.exp(go[m])) <= 1e-5 * np.exp(go[m])).all(), \
            np.max(np.abs(g[m] - go[m]))
    finally:
        ctx.close()
