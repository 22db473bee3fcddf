"""The measured MI355X profiles: layout of the stored dataset and of the
batches built from it, and the oracle running end to end on them."""
import numpy as np

from oracle import plain as P
from paper_1910_07776_amd.profiling import dataset as R


def test_dataset_layout():
    d = R.load()
    assert d["counters"].shape == (2 * 3 * 3 * 64, 18) and len(d["names"]) == 18
    assert (d["counters"] >= 0).all() and (d["cycles"] > 0).all()
    # every (program, input, run) sweep holds the 64 versions once
    for p, i, r in R.sweeps():
        sel = (d["program"] == p) & (d["input"] == i) & (d["run"] == r)
        assert sorted(d["version"][sel]) == list(range(64))


def test_batch_layout_and_oracle_end_to_end():
    d = R.load()
    b = R.batch(d, R.sweeps(0, inputs=(1,)))
    assert b.K == 3 and b.N == 192 and (b.counters >= 1).all()
    assert list(b.row_off) == [0, 64, 128, 192] and list(b.opt_ids[:6]) == list(range(6))
    model = P.fit(b, 6)
    assert (model["counts"] == 3 * 32).all()
    grid, table, sug = P.run(model, b)
    assert np.isfinite(table).all() and len(sug) == 3
    # the measured log-speedups the model learns from are the cycle ratios
    y = np.log(b.cycles[0]) - np.log(b.cycles[1])
    assert np.isclose(y, np.log(d["cycles"][(d["program"] == 0) & (d["input"] == 1) & (d["run"] == 0)][0:2]).dot([1, -1]))
