"""The seeded synthetic world: layout, regenerability, the stored digests and
the oracle's outputs on the 2-kernel world.  CPU only."""
import hashlib
import json
import os

import numpy as np

from synthgen import make_batch, kernel_layout
from oracle import plain as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_outputs.json")))


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_layout_and_truth():
    b = make_batch(5, range(40), 16, 10, brange=(0, 6))
    assert b.row_off[0] == 0 and b.opt_off[0] == 0
    assert (np.diff(b.row_off) == 1 << b.nopts.astype(np.int64)).all()
    assert (np.diff(b.opt_off) == b.nopts).all()
    for k in range(b.K):
        O = b.kernel_opts(k)
        assert (np.diff(O) > 0).all() and (O < 10).all()
        r = b.kernel_rows(k)
        assert b.truth[r][0] == 0.0
        # the true log-speedup is encoded in the cycle counts
        np.testing.assert_allclose(np.log(b.cycles[r][0]) - np.log(b.cycles[r]),
                                   b.truth[r], atol=2e-6)
    assert (b.counters > 0).all() and (b.cycles > 0).all()


def test_kernels_regenerate_alone():
    b = make_batch(1910, range(300), 128, 10, brange=(4, 10))
    for k in (0, 17, 299):
        one = make_batch(1910, [k], 128, 10, brange=(4, 10))
        r = b.kernel_rows(k)
        np.testing.assert_array_equal(b.counters[r], one.counters)
        np.testing.assert_array_equal(b.cycles[r], one.cycles)
        np.testing.assert_array_equal(b.kernel_opts(k), one.opt_ids)


def test_ragged_range_and_layout_helper():
    b = make_batch(1910, range(2000), 8, 10, brange=(4, 10))
    assert b.nopts.min() == 4 and b.nopts.max() == 10
    ro, oo = kernel_layout(b.nopts)
    np.testing.assert_array_equal(ro, b.row_off)
    np.testing.assert_array_equal(oo, b.opt_off)


def test_lognormal_counter_scale():
    b = make_batch(1910, range(200), 32, 6)
    base = b.counters[b.row_off[:-1]]
    sd = np.log(base).std(axis=0)
    assert 0.4 < sd.mean() < 0.6            # sigma 0.5 across kernels


def test_stored_digests():
    b = make_batch(1910, range(2), 40, 6, dtype=np.float64)
    assert digest(b.counters, b.cycles, b.truth) == GOLD["generator_2x64x40_f64"]
    r = make_batch(1910, range(64), 128, 10, brange=(4, 10))
    assert digest(r.nopts, r.opt_ids, r.counters, r.cycles) == GOLD["generator_ragged64_f32"]


def test_oracle_stored_outputs_2_kernel_world():
    b = make_batch(1910, range(2), 40, 6, dtype=np.float64)
    folds = P.leave_one_kernel_out(b, 6)
    for f, g in zip(folds, GOLD["loko_2x64x40"]):
        np.testing.assert_allclose(f["model"]["W"], np.array(g["W"]), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(f["table"], np.array(g["table"]), rtol=1e-9, atol=1e-12)
        assert [i for i, _ in f["suggestions"][0]] == [i for i, _ in g["suggestions"]]
