"""GPU parity of the plain scoring path against the FP64 oracle, called
through the C ABI.

Tolerances: scores are compared on the speedup scale e^L,
|e^L_gpu - e^L_oracle| <= rtol * e^L_oracle, with rtol 1e-5 for the FP32
path and 1e-8 for the FP64 path; suggestion lists must be identical except
where the oracle's scores are within that tolerance of each other, of the
threshold or of the n-th place (oracle.checks.check_list).  Generic ranking of
given scores is integer work and must be bit-exact.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import plain as P
from oracle.checks import check_list
from synthgen import make_batch

pytestmark = pytest.mark.gpu

RTOL32 = 1e-5
RTOL64 = 1e-8
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def G():
    from paper_1910_07776_amd import plain
    return plain


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def plan_of(G, ctx, b, D, dtype=torch.float32):
    return G.Plan(ctx, b.nopts, b.opt_ids, b.E if hasattr(b, "E") else b.counters.shape[1], D, dtype)


def gpu_inputs(b, dtype=torch.float32):
    return to_dev(b.counters, dtype), to_dev(b.cycles, dtype)


def assert_scores(got, want, rtol, what):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    assert (nan_g == nan_w).all(), f"{what}: NaN pattern differs"
    m = ~nan_w
    err = np.abs(np.exp(got[m]) - np.exp(want[m])) / np.exp(want[m])
    worst = float(err.max()) if err.size else 0.0
    assert worst <= rtol, f"{what}: worst relative speedup error {worst:.3e} > {rtol:g}"
    return worst


def check_suggestions(idx, score, count, table_ora, row_off, tau, n, tol):
    idx, score, count = idx.cpu().numpy(), score.cpu().numpy(), count.cpu().numpy()
    bad = []
    for k in range(len(count)):
        c = int(count[k])
        assert (idx[k, c:] == -1).all() and np.isnan(score[k, c:]).all()
        seg = table_ora[row_off[k]:row_off[k + 1]]
        errs = check_list(idx[k, :c], score[k, :c], seg, tau, n, tol, first=1)
        if errs:
            bad.append((k, errs))
    assert not bad, bad[:5]


# ------------------------------------------------------------------------
def test_512_kernels_fit_predict_suggest(G, ctx):
    """512 kernels x 64 versions x 128 events, FP32; fit on 512 other kernels."""
    tr = make_batch(1910, range(10 ** 6, 10 ** 6 + 512), 128, 6)
    te = make_batch(1910, range(512), 128, 6)
    om = P.fit(tr, 6)
    ogrid, otab, osug = P.run(om, te)

    ptr = plan_of(G, ctx, tr, 6)
    G.fit(ctx, ptr, *gpu_inputs(tr))
    G.sync(ctx)
    m = ctx.model_get()
    np.testing.assert_allclose(m["mu"], om["mu"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(m["sigma"], om["sigma"], rtol=1e-12)
    np.testing.assert_allclose(m["W"], om["W"], rtol=1e-9, atol=1e-11)
    assert (m["counts"] == om["counts"]).all()

    pte = plan_of(G, ctx, te, 6)
    c, cy = gpu_inputs(te)
    idx, score, count, table = G.suggest(ctx, pte, c, cy)
    tab, grid = G.predict(ctx, pte, c, cy, grid=True)
    G.sync(ctx)
    assert_scores(table.cpu().numpy(), otab, RTOL32, "table")
    assert torch.equal(table, tab)
    assert_scores(grid.cpu().numpy(), ogrid, RTOL32, "grid")
    check_suggestions(idx, score, count, otab, te.row_off, P.TAU, 3, RTOL32)
    # the launch shape the benchmark times (its tuning-database entry for this
    # plan) gives the same bits
    from paper_1910_07776_amd import tuning
    db = tuning.TuneCache(os.path.join(os.path.dirname(HERE), "paper_1910_07776_amd", "tuning_db.json"))
    key = tuning.plan_key(pte, 3)
    assert key in db, key
    if "items" in db[key]:
        pte.set_items(db[key]["items"])
    pte.set_launch(db[key]["waves"], db[key]["unroll"], 0)
    again = G.suggest(ctx, pte, c, cy)
    G.sync(ctx)
    for x, y in zip((idx, score, count, table), again):
        assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0))


def test_two_kernel_cross_program_folds_fp64(G, ctx):
    """2 kernels x 64 versions x 40 events, FP64: fit on one kernel, score the
    other (Section 5's train-on-one-program, test-on-another protocol)."""
    b = make_batch(1910, range(2), 40, 6, dtype=np.float64)
    folds = P.leave_one_kernel_out(b, 6)
    for k, f in enumerate(folds):
        tr = P.SubBatch(b, [1 - k])
        te = f["test"]
        ptr = G.Plan(ctx, tr.nopts, tr.opt_ids, 40, 6, torch.float64)
        G.fit(ctx, ptr, to_dev(tr.counters), to_dev(tr.cycles))
        G.sync(ctx)
        m = ctx.model_get()
        np.testing.assert_allclose(m["W"], f["model"]["W"], rtol=1e-8, atol=1e-9)
        pte = G.Plan(ctx, te.nopts, te.opt_ids, 40, 6, torch.float64)
        idx, score, count, table = G.suggest(ctx, pte, to_dev(te.counters), to_dev(te.cycles))
        _, grid = G.predict(ctx, pte, to_dev(te.counters), to_dev(te.cycles), grid=True)
        G.sync(ctx)
        assert_scores(table.cpu().numpy(), f["table"], RTOL64, "table")
        assert_scores(grid.cpu().numpy(), f["grid"], RTOL64, "grid")
        check_suggestions(idx, score, count, f["table"], te.row_off, P.TAU, 3, RTOL64)


@pytest.fixture(scope="module")
def ragged(G, ctx):
    """A ragged batch with every kernel size 0..12 optimisations (1-4096
    versions), fitted on another draw of the same world."""
    tr = make_batch(77, range(5000, 5000 + 256), 128, 12, brange=(0, 12))
    te = make_batch(77, range(256), 128, 12, brange=(0, 12))
    om = P.fit(tr, 12)
    ptr = plan_of(G, ctx, tr, 12)
    G.fit(ctx, ptr, *gpu_inputs(tr))
    G.sync(ctx)
    return tr, te, om


def test_ragged_all_sizes(G, ctx, ragged):
    tr, te, om = ragged
    assert te.nopts.min() == 0 and te.nopts.max() == 12
    ogrid, otab, osug = P.run(om, te)
    pte = plan_of(G, ctx, te, 12)
    c, cy = gpu_inputs(te)
    idx, score, count, table = G.suggest(ctx, pte, c, cy)
    _, grid = G.predict(ctx, pte, c, cy, grid=True)
    G.sync(ctx)
    assert_scores(table.cpu().numpy(), otab, RTOL32, "table")
    assert_scores(grid.cpu().numpy(), ogrid, RTOL32, "grid")
    check_suggestions(idx, score, count, otab, te.row_off, P.TAU, 3, RTOL32)


def test_batching_invariance_bit_exact(G, ctx, ragged):
    tr, te, om = ragged
    pte = plan_of(G, ctx, te, 12)
    c, cy = gpu_inputs(te)
    idx, score, count, table = G.suggest(ctx, pte, c, cy)
    picks = [int(np.argmin(te.nopts)), int(np.argmax(te.nopts))] + \
        [int(np.flatnonzero(te.nopts == b)[0]) for b in (1, 5, 6, 7, 9)]
    for k in picks:
        one = P.SubBatch(te, [k])
        p1 = G.Plan(ctx, one.nopts, one.opt_ids, 128, 12)
        i1, s1, c1, t1 = G.suggest(ctx, p1, to_dev(one.counters), to_dev(one.cycles))
        r0, r1 = te.row_off[k], te.row_off[k + 1]
        assert torch.equal(t1, table[r0:r1]), k
        assert torch.equal(i1[0], idx[k]) and torch.equal(c1[0], count[k]), k
        assert torch.equal(torch.nan_to_num(s1[0], nan=-7.0), torch.nan_to_num(score[k], nan=-7.0)), k


def test_deterministic_runs(G, ctx, ragged):
    tr, te, om = ragged
    pte = plan_of(G, ctx, te, 12)
    c, cy = gpu_inputs(te)
    a = G.suggest(ctx, pte, c, cy)
    b = G.suggest(ctx, pte, c, cy)
    for x, y in zip(a, b):
        assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0))
    w0 = ctx.model_get()["W"]
    ptr = plan_of(G, ctx, tr, 12)
    G.fit(ctx, ptr, *gpu_inputs(tr))
    G.sync(ctx)
    assert np.array_equal(ctx.model_get()["W"], w0)


def test_load_features_stats_and_z(G):
    ctx = G.Context(0)   # own context: new statistics invalidate a fitted model
    b = make_batch(31, range(300), 128, 6)
    x = P.features(b.counters, b.cycles)
    mu, sg = P.column_stats(x)
    p = plan_of(G, ctx, b, 6)
    c, cy = gpu_inputs(b)
    z = G.load_features(ctx, p, c, cy, fit_stats=True, apply=True)
    G.sync(ctx)
    m = ctx.model_get()
    np.testing.assert_allclose(m["mu"], mu, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(m["sigma"], sg, rtol=1e-12)
    zo = P.standardize(x, mu, sg)
    # FP32 log of values up to e^17 (about 1 ulp, 1e-6) and FP32 mean/scale
    np.testing.assert_allclose(z.cpu().numpy(), zo, rtol=0, atol=3e-5)
    ctx.close()


def test_generic_rank_bit_exact(G, ctx):
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 300, size=200)
    lens[:3] = [0, 1, 64]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    for dt, npdt in ((torch.float32, np.float32), (torch.float64, np.float64)):
        s = np.round(rng.normal(0.05, 0.08, size=off[-1]), 3).astype(npdt)
        s[rng.random(off[-1]) < 0.02] = np.nan
        for n in (1, 3, 8):
            for skip in (0, 1):
                tau = float(npdt(P.TAU))
                idx, sc, cnt = G.rank_suggest(ctx, to_dev(s), to_dev(off), n=n, tau=tau, skip_head=skip)
                idx, sc, cnt = idx.cpu().numpy(), sc.cpu().numpy(), cnt.cpu().numpy()
                for i in range(len(lens)):
                    want = P.rank(s[off[i]:off[i + 1]].astype(np.float64), tau, n, first=skip)
                    assert cnt[i] == len(want)
                    assert [int(v) for v in idx[i, :cnt[i]]] == [j for j, _ in want]
                    assert np.array_equal(sc[i, :cnt[i]].astype(np.float64), [v for _, v in want])
                    assert (idx[i, cnt[i]:] == -1).all()


def test_per_version_ranking_of_the_grid(G, ctx, ragged):
    """The tool's own output form: for one profiled version, the best single
    optimisations above the threshold (rank over grid rows)."""
    tr, te, om = ragged
    pte = plan_of(G, ctx, te, 12)
    _, grid = G.predict(ctx, pte, *gpu_inputs(te), grid=True)
    N, Bm = grid.shape
    off = torch.arange(0, N + 1, dtype=torch.int64, device="cuda") * Bm
    idx, sc, cnt = G.rank_suggest(ctx, grid.reshape(-1).contiguous(), off, n=3, tau=float(np.float32(P.TAU)))
    g = grid.cpu().numpy().astype(np.float64)
    want = P.suggest_rows(g, float(np.float32(P.TAU)), 3)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for r in range(0, N, 7):
        assert [int(v) for v in idx[r, :cnt[r]]] == [j for j, _ in want[r]]


def test_empty_and_zero_option_batches(G, ctx, ragged):
    p0 = G.Plan(ctx, np.zeros(0, np.int32), np.zeros(0, np.int32), 128, 12)
    c = torch.empty((0, 128), device="cuda")
    cy = torch.empty(0, device="cuda")
    idx, sc, cnt, tab = G.suggest(ctx, p0, c, cy)
    assert idx.shape == (0, 3) and tab.shape == (0,)
    b = make_batch(3, range(10), 128, 12, brange=(0, 0))
    p = plan_of(G, ctx, b, 12)
    idx, sc, cnt, tab = G.suggest(ctx, p, *gpu_inputs(b))
    G.sync(ctx)
    assert (tab.cpu() == 0).all() and (cnt.cpu() == 0).all() and (idx.cpu() == -1).all()


def test_errors(G, ctx, ragged):
    from paper_1910_07776_amd._abi import SuggError
    tr, te, om = ragged
    b = make_batch(77, range(40), 128, 12, brange=(3, 6))
    p = plan_of(G, ctx, b, 12)
    c, cy = gpu_inputs(b)
    c[5, 3] = 0.0
    G.suggest(ctx, p, c, cy)
    with pytest.raises(SuggError) as e:
        G.sync(ctx)
    assert e.value.name == "SUGG_E_BAD_COUNTER"
    G.sync(ctx)  # cleared
    c, cy = gpu_inputs(b)
    cy[7] = float("nan")
    G.predict(ctx, p, c, cy)
    with pytest.raises(SuggError) as e:
        G.sync(ctx)
    assert e.value.name == "SUGG_E_BAD_COUNTER"
    with pytest.raises(SuggError) as e:
        G.Plan(ctx, np.array([2], np.int32), np.array([3, 1], np.int32), 128, 12)
    assert e.value.name == "SUGG_E_SHAPE"
    with pytest.raises(SuggError) as e:
        G.Plan(ctx, np.array([13], np.int32), np.arange(13, dtype=np.int32), 128, 14)
    assert e.value.name == "SUGG_E_SHAPE"
    with pytest.raises(SuggError) as e:
        G.rank_suggest(ctx, torch.zeros(4, device="cuda"), torch.tensor([0, 4], device="cuda"), n=9)
    assert e.value.name == "SUGG_E_ARG"
    # a model trained without optimisation id 13 cannot score it
    q = G.Plan(ctx, np.array([1], np.int32), np.array([13], np.int32), 128, 14)
    with pytest.raises(SuggError) as e:
        G.predict(ctx, q, torch.ones((2, 128), device="cuda"), torch.ones(2, device="cuda"))
    assert e.value.name == "SUGG_E_UNTRAINED_OPT"
    fresh = G.Context(0)
    with pytest.raises(SuggError) as e:
        G.predict(fresh, G.Plan(fresh, b.nopts, b.opt_ids, 128, 12), *gpu_inputs(b))
    assert e.value.name == "SUGG_E_STATE"
    fresh.close()


def test_model_checkpoint_roundtrip(G, ctx, ragged):
    tr, te, om = ragged
    pte = plan_of(G, ctx, te, 12)
    c, cy = gpu_inputs(te)
    a = G.suggest(ctx, pte, c, cy)
    m = ctx.model_get()
    other = G.Context(0)
    other.model_set(m)
    p2 = plan_of(G, other, te, 12)
    b = G.suggest(other, p2, c, cy)
    for x, y in zip(a, b):
        assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0))
    other.close()


def test_ragged_16384_kernels_full_size(G):
    """16,384 kernels with 4-10 of 10 optimisations (4.8M versions, 128
    events): the GPU fit against the oracle's stored fit, and the scoring
    launch the benchmark times against one oracle run over every kernel
    (table element by element, every suggestion list)."""
    ctx = G.Context(0)   # own context: the shared one keeps the fixture's model
    gold = json.load(open(os.path.join(HERE, "golden", "ragged16384_model.json")))
    om = {k: np.asarray(gold[k]) for k in ("mu", "sigma", "W", "counts")}
    t0, t1 = gold["train_ids"]
    tr = make_batch(1910, range(t0, t1), 128, 10, brange=(4, 10))
    ptr = plan_of(G, ctx, tr, 10)
    G.fit(ctx, ptr, *gpu_inputs(tr))
    G.sync(ctx)
    m = ctx.model_get()
    np.testing.assert_allclose(m["W"], om["W"], rtol=1e-9, atol=1e-11)
    del tr, ptr
    te = make_batch(1910, range(16384), 128, 10, brange=(4, 10))
    pte = plan_of(G, ctx, te, 10)
    # in the launch shape the benchmark times (its tuning-database entry)
    from paper_1910_07776_amd import tuning
    db = tuning.TuneCache(os.path.join(os.path.dirname(HERE), "paper_1910_07776_amd", "tuning_db.json"))
    key = tuning.plan_key(pte, 3)
    assert key in db, key
    if "items" in db[key]:
        pte.set_items(db[key]["items"])
    pte.set_launch(db[key]["waves"], db[key]["unroll"], 0)
    idx, score, count, table = G.suggest(ctx, pte, *gpu_inputs(te))
    G.sync(ctx)
    table, idx, score, count = (t.cpu().numpy() for t in (table, idx, score, count))
    for c0 in range(0, 16384, 2048):
        sub = P.SubBatch(te, range(c0, c0 + 2048))
        _, tab, _ = P.run(om, sub)
        r0, r1 = te.row_off[c0], te.row_off[c0 + 2048]
        assert_scores(table[r0:r1], tab, RTOL32, f"kernels {c0}..{c0 + 2047}")
        for k in range(c0, c0 + 2048):
            seg = tab[sub.row_off[k - c0]:sub.row_off[k - c0 + 1]]
            errs = check_list(idx[k, :count[k]], score[k, :count[k]], seg, P.TAU, 3, RTOL32, first=1)
            assert not errs, (k, errs)
        print(f"kernels {c0}..{c0 + 2047}: tables and lists match the oracle", flush=True)
    del pte
    ctx.close()


def test_launch_shapes_and_persistent_queue_bit_identical(G, ctx, ragged):
    """Every launch shape the autotuner may pick, and a forced small grid that
    makes workgroups pull items from the atomic counter (relaunched so the
    counter's self re-arm is exercised), give bit-identical results."""
    tr, te, om = ragged
    pte = plan_of(G, ctx, te, 12)
    c, cy = gpu_inputs(te)
    ref = [t.clone() for t in G.suggest(ctx, pte, c, cy)]
    shapes = [(w, u, 0) for w in (1, 2, 4, 8) for u in (1, 2, 4)] + [(4, 2, 3), (2, 4, 7), (8, 1, 1)] + \
        [(4, -1, 0), (4, -2, 0), (4, -4, 0)]   # the streaming form
    for w, u, g in shapes:
        pte.set_launch(w, u, g)
        for _ in range(2):
            out = G.suggest(ctx, pte, c, cy)
            for x, y in zip(ref, out):
                assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0),
                                   torch.nan_to_num(y.double(), nan=-7.0)), (w, u, g)
    G.sync(ctx)
    cfg = G.autotune(ctx, pte, c, cy, reps=2)
    assert cfg["waves"] in (2, 4, 8) and cfg["unroll"] in (1, 2, 4, -1, -2, -4)
    assert cfg["items"] in (64, 128, 256, 512, 1024)
    assert len(cfg["times_ms"]) == 60 and all(v > 0 for v in cfg["times_ms"].values())
    assert pte.get_items() == cfg["items"]
    # every item size gives the same bits as the default one
    for rows in (16, 128, 1024, 4096):
        pte.set_items(rows)
        pte.set_launch(4, 1, 0)
        out = G.suggest(ctx, pte, c, cy)
        for x, y in zip(ref, out):
            assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0)), rows
        pte.set_launch(4, 2, 3)   # persistent: items taken from the queue, the next one's rows prefetched
        out = G.suggest(ctx, pte, c, cy)
        for x, y in zip(ref, out):
            assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0)), rows
    G.sync(ctx)


def test_graph_replays_match_eager(G, ctx, ragged):
    """A captured scoring pass replayed several times, with eager work and new
    inputs copied into its buffers between replays."""
    tr, te, om = ragged
    te2 = make_batch(77, range(256), 128, 12, brange=(0, 12))   # same structure
    other = make_batch(77, range(9000, 9256), 128, 12, brange=(0, 12))
    pte = plan_of(G, ctx, te, 12)
    c, cy = gpu_inputs(te)
    n = ctx.params["n_suggest"]
    out = {"idx": torch.empty((te.K, n), dtype=torch.int32, device="cuda"),
           "score": torch.empty((te.K, n), device="cuda"),
           "count": torch.empty(te.K, dtype=torch.int32, device="cuda"),
           "table": torch.empty(te.N, device="cuda")}
    pte.set_launch(4, 2, 5)   # persistent mode: the counter re-arms itself each replay
    g = G.Graph(ctx)
    with g.capture():
        G.suggest(ctx, pte, c, cy, out=out)
    eager = [t.clone() for t in G.suggest(ctx, pte, c, cy)]
    for rep in range(4):
        if rep == 2:
            # new inputs of the same structure, copied into the captured buffers
            c2, cy2 = gpu_inputs(te2)
            c.copy_(c2)
            cy.copy_(cy2)
            eager = [t.clone() for t in G.suggest(ctx, pte, c, cy)]
        g.launch()
        torch.cuda.synchronize()
        for x, y in zip(eager, (out["idx"], out["score"], out["count"], out["table"])):
            assert torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0)), rep
        # unrelated eager work between replays
        po = plan_of(G, ctx, other, 12)
        G.suggest(ctx, po, *gpu_inputs(other))
    G.sync(ctx)
    g.close()


def _same(x, y):
    return torch.equal(torch.nan_to_num(x.double(), nan=-7.0), torch.nan_to_num(y.double(), nan=-7.0))


@pytest.mark.parametrize("E,B,dtype,n", [(128, 6, torch.float32, 3), (128, 6, torch.float64, 3),
                                         (37, 5, torch.float32, 8), (200, 4, torch.float64, 3),
                                         (64, 3, torch.float32, 2), (128, 1, torch.float32, 3)])
def test_split_form_bit_identical_to_fused(G, E, B, dtype, n):
    """The split form (16 versions per workgroup, the last of a kernel's
    workgroups composing and ranking) against the fused kernel, bit for bit,
    over repeated launches (the arrival counters re-arm themselves) and graph
    replays with eager work in between."""
    npdt = np.float32 if dtype == torch.float32 else np.float64
    tr = make_batch(88, range(3000, 3064), E, B, dtype=npdt)
    te = make_batch(88, range(200), E, B, dtype=npdt)
    c_ = G.Context(0, n_suggest=n)
    try:
        G.fit(c_, plan_of(G, c_, tr, B, dtype), *gpu_inputs(tr, dtype))
        pte = plan_of(G, c_, te, B, dtype)
        c, cy = gpu_inputs(te, dtype)
        pte.set_launch(4, 1, 0)
        ref = [t.clone() for t in G.suggest(c_, pte, c, cy)]
        ref_tab = G.predict(c_, pte, c, cy)[0].clone()
        pte.set_launch(4, 0, 0)
        assert pte.get_launch()["unroll"] == 0
        for _ in range(3):
            out = G.suggest(c_, pte, c, cy)
            assert all(_same(x, y) for x, y in zip(ref, out))
        assert _same(G.predict(c_, pte, c, cy)[0], ref_tab)
        # the grid form falls back to the fused kernel and agrees too
        tab_g, _ = G.predict(c_, pte, c, cy, grid=True)
        assert _same(tab_g, ref_tab)
        bufs = {"idx": torch.empty((te.K, n), dtype=torch.int32, device="cuda"),
                "score": torch.empty((te.K, n), dtype=dtype, device="cuda"),
                "count": torch.empty(te.K, dtype=torch.int32, device="cuda"),
                "table": torch.empty(te.N, dtype=dtype, device="cuda")}
        g = G.Graph(c_)
        with g.capture():
            G.suggest(c_, pte, c, cy, out=bufs)
        for _ in range(3):
            for t in bufs.values():
                t.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert all(_same(x, bufs[k]) for x, k in zip(ref, ("idx", "score", "count", "table")))
            G.suggest(c_, pte, c, cy)   # eager launches between replays
        G.sync(c_)
        g.close()
    finally:
        c_.close()


def test_split_form_512_kernels_against_oracle(G):
    """The headline batch (512 kernels x 64 versions x 128 FP32 events) in the
    split form against the oracle; the autotuner includes the form."""
    tr = make_batch(1910, range(10 ** 6, 10 ** 6 + 512), 128, 6)
    te = make_batch(1910, range(512), 128, 6)
    om = P.fit(tr, 6)
    _, otab, _ = P.run(om, te)
    c_ = G.Context(0)
    try:
        G.fit(c_, plan_of(G, c_, tr, 6), *gpu_inputs(tr))
        pte = plan_of(G, c_, te, 6)
        c, cy = gpu_inputs(te)
        pte.set_launch(4, 0, 0)
        idx, score, count, table = G.suggest(c_, pte, c, cy)
        G.sync(c_)
        assert_scores(table.cpu().numpy(), otab, RTOL32, "table")
        check_suggestions(idx, score, count, otab, te.row_off, P.TAU, 3, RTOL32)
        cfg = G.autotune(c_, pte, c, cy, reps=2)
        assert len(cfg["times_ms"]) == 61 and cfg["times_ms"]["split"] > 0
        assert cfg["unroll"] in (0, 1, 2, 4, -1, -2, -4)
    finally:
        c_.close()


@pytest.mark.parametrize("E,dtype,D,brange", [(1, torch.float32, 4, (0, 4)), (37, torch.float32, 6, (0, 6)),
                                              (64, torch.float64, 5, (2, 5)), (200, torch.float32, 8, (0, 8)),
                                              (256, torch.float32, 6, None), (256, torch.float64, 10, (4, 10))])
def test_event_counts_against_oracle(G, E, dtype, D, brange):
    """The fused path over the event counts the kernels are built for (one
    event up to the maximum of 256; chunked and scalar loads), both dtypes,
    mixed and uniform B: table, grid and suggestions against the oracle."""
    npdt = np.float32 if dtype == torch.float32 else np.float64
    rtol = RTOL32 if dtype == torch.float32 else RTOL64
    tr = make_batch(91, range(7000, 7048), E, D, brange=brange, dtype=npdt)
    te = make_batch(91, range(60), E, D, brange=brange, dtype=npdt)
    om = P.fit(tr, D)
    ogrid, otab, _ = P.run(om, te)
    c_ = G.Context(0)
    try:
        G.fit(c_, plan_of(G, c_, tr, D, dtype), *gpu_inputs(tr, dtype))
        pte = plan_of(G, c_, te, D, dtype)
        c, cy = gpu_inputs(te, dtype)
        idx, score, count, table = G.suggest(c_, pte, c, cy)
        tab, grid = G.predict(c_, pte, c, cy, grid=True)
        G.sync(c_)
        assert_scores(table.cpu().numpy(), otab, rtol, f"table E={E}")
        assert torch.equal(table, tab)
        g = grid.cpu().numpy()[:, :ogrid.shape[1]]
        assert_scores(g, ogrid, rtol, f"grid E={E}")
        check_suggestions(idx, score, count, otab, te.row_off, P.TAU, 3, rtol)
    finally:
        c_.close()
