"""Writes the stored expected values under tests/golden/.

Runs only the seeded generator and the FP64 oracle:
    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synthgen import make_batch  # noqa: E402
from oracle import plain as P  # noqa: E402


RAGGED_TRAIN0 = 1_000_000


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    out = {}
    # the 2-kernel, 64-version, 40-event FP64 world (seed 1910)
    b = make_batch(1910, range(2), 40, 6, dtype=np.float64)
    out["generator_2x64x40_f64"] = digest(b.counters, b.cycles, b.truth)
    r = make_batch(1910, range(64), 128, 10, brange=(4, 10))
    out["generator_ragged64_f32"] = digest(r.nopts, r.opt_ids, r.counters, r.cycles)
    folds = P.leave_one_kernel_out(b, 6)
    out["loko_2x64x40"] = [{
        "W": f["model"]["W"].tolist(),
        "table": f["table"].tolist(),
        "suggestions": [[int(i), float(v)] for i, v in f["suggestions"][0]],
    } for f in folds]
    with open(os.path.join(HERE, "oracle_outputs.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    # the oracle's model fitted on the ragged training draw of 16,384 kernels
    # (4-10 optimisations of 10, 128 events, FP32 counters)
    tr = make_batch(1910, range(RAGGED_TRAIN0, RAGGED_TRAIN0 + 16384), 128, 10, brange=(4, 10))
    m = P.fit(tr, 10)
    with open(os.path.join(HERE, "ragged16384_model.json"), "w") as fh:
        json.dump({"train_ids": [RAGGED_TRAIN0, RAGGED_TRAIN0 + 16384], "E": 128, "D": 10,
                   "mu": m["mu"].tolist(), "sigma": m["sigma"].tolist(), "W": m["W"].tolist(),
                   "counts": m["counts"].tolist(), "rows": int(tr.N)}, fh)


if __name__ == "__main__":
    main()
