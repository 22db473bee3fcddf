"""Checkpoints: every fitted model saved, loaded into a fresh context, and
predicting bit for bit as before; surrogate training resumed from a
checkpoint equal bit for bit to the uninterrupted run."""
import numpy as np
import pytest
import torch

from synthgen import make_batch

pytestmark = pytest.mark.gpu

E, D = 64, 8


@pytest.fixture(scope="module")
def G():
    from paper_1910_07776_amd import plain
    return plain


@pytest.fixture(scope="module")
def CK():
    from paper_1910_07776_amd import checkpoint
    return checkpoint


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def data():
    tr = make_batch(71, range(3000, 3040), E, D, brange=(3, 7))
    te = make_batch(71, range(24), E, D, brange=(2, 7))
    return tr, te


def same(a, b):
    return torch.equal(torch.nan_to_num(a.double(), nan=-7.0), torch.nan_to_num(b.double(), nan=-7.0))


def test_plain_checkpoint(G, CK, data, tmp_path):
    tr, te = data
    c1, c2 = G.Context(0), G.Context(0)
    G.fit(c1, G.Plan(c1, tr.nopts, tr.opt_ids, E, D), dev(tr.counters), dev(tr.cycles))
    CK.save_plain(c1, str(tmp_path / "plain.safetensors"))
    CK.load_plain(c2, str(tmp_path / "plain.safetensors"))
    outs = []
    for c in (c1, c2):
        p = G.Plan(c, te.nopts, te.opt_ids, E, D)
        outs.append(G.suggest(c, p, dev(te.counters), dev(te.cycles)))
        G.sync(c)
    for x, y in zip(*outs):
        assert same(x, y)
    with pytest.raises(ValueError):
        CK.load_m5p(c2, str(tmp_path / "plain.safetensors"))   # another kind
    c1.close()
    c2.close()


def test_m5p_checkpoint(G, CK, data, tmp_path):
    tr, te = data
    c1, c2 = G.Context(0), G.Context(0)
    G.m5p_fit(c1, G.Plan(c1, tr.nopts, tr.opt_ids, E, D), dev(tr.counters), dev(tr.cycles))
    CK.save_m5p(c1, str(tmp_path / "m5p.safetensors"))
    CK.load_m5p(c2, str(tmp_path / "m5p.safetensors"))
    for o in range(D):
        a, b = G.m5p_tree(c1, o), G.m5p_tree(c2, o)
        for k in a:
            assert np.array_equal(np.nan_to_num(a[k], nan=-7.0), np.nan_to_num(b[k], nan=-7.0)), (o, k)
    for dtype in (torch.float32, torch.float64):
        outs = []
        for c in (c1, c2):
            p = G.Plan(c, te.nopts, te.opt_ids, E, D, dtype=dtype)
            outs.append(G.m5p_suggest(c, p, dev(te.counters).to(dtype), dev(te.cycles).to(dtype)))
            G.sync(c)
        for x, y in zip(*outs):
            assert same(x, y)
    # a damaged tree is refused and the previous model stays
    m = CK.m5p_export(c2)
    bad = dict(m)
    bad["left"] = m["left"].copy()
    inner = np.nonzero(m["feat"] >= 0)[0]
    bad["left"][inner[0]] = inner[0]            # a node its own child
    with pytest.raises(Exception):
        CK.m5p_import(c2, bad)
    bad = dict(m)
    bad["leaf"] = m["leaf"].copy()
    leaves = np.nonzero(m["feat"] < 0)[0]
    bad["leaf"][leaves[1]] = bad["leaf"][leaves[0]]   # one leaf model used twice
    with pytest.raises(Exception):
        CK.m5p_import(c2, bad)
    bad = dict(m)
    bad["isg"] = m["isg"].copy()
    bad["isg"][3] = np.nan
    with pytest.raises(Exception):
        CK.m5p_import(c2, bad)
    assert np.array_equal(CK.m5p_export(c2)["lw"], m["lw"])
    c1.close()
    c2.close()


def test_ibk_checkpoint(G, CK, data, tmp_path):
    tr, te = data
    c1, c2 = G.Context(0), G.Context(0)
    ptr = G.Plan(c1, tr.nopts, tr.opt_ids, E, D)
    c, cy = dev(tr.counters), dev(tr.cycles)
    G.ibk_fit(c1, ptr, c, cy, 5)
    CK.save_ibk(str(tmp_path / "ibk.safetensors"), ptr, c, cy, 5)
    keep = CK.load_ibk(c2, str(tmp_path / "ibk.safetensors"))
    outs = []
    for cx in (c1, c2):
        p = G.Plan(cx, te.nopts, te.opt_ids, E, D)
        outs.append(G.ibk_suggest(cx, p, dev(te.counters), dev(te.cycles)))
        G.sync(cx)
    for x, y in zip(*outs):
        assert same(x, y)
    del keep
    c1.close()
    c2.close()


def test_surrogate_resume_is_bit_exact(CK, tmp_path):
    from paper_1910_07776_amd import plain as G
    from paper_1910_07776_amd.surrogate import MLP
    ctx = G.Context(0)
    rng = np.random.default_rng(5)
    X = torch.tensor(rng.normal(size=(6, 512, 128)), dtype=torch.float32, device="cuda")
    Y = torch.tensor(rng.normal(size=(6, 512, 64)) * 0.1, dtype=torch.float32, device="cuda")
    full = MLP(ctx, 128, 512, 64, max_batch=512, seed=3)
    for s in range(6):
        full.train_step(X[s], Y[s], lr=1e-3)
    part = MLP(ctx, 128, 512, 64, max_batch=512, seed=3)
    for s in range(3):
        part.train_step(X[s], Y[s], lr=1e-3)
    CK.save_surrogate(part, str(tmp_path / "mlp.safetensors"))
    del part
    res = CK.load_surrogate(ctx, str(tmp_path / "mlp.safetensors"))
    assert res.step == 3
    for s in range(3, 6):
        res.train_step(X[s], Y[s], lr=1e-3)
    G.sync(ctx)
    assert torch.equal(full.params, res.params)
    assert torch.equal(full.m, res.m) and torch.equal(full.v, res.v)
    assert full.step == res.step == 6
    ctx.close()
