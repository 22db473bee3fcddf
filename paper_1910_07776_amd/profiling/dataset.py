"""The measured MI355X profiles (mi355x_versions.npz, written by collect.py
from the versions.hip programs) as batches in the library's layout.

A "kernel" of a batch is one profiled sweep: one program on one input in one
run, its 64 versions in subset order (bit b = optimisation b, the same six
global ids in both programs).  Counters are the measured event counts plus
one, so an event that did not occur (LDS instructions in a version without
LDS staging) gives a finite feature ln(1 / cycles) instead of ln 0.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mi355x_versions.npz")
OPTS = ("FAST", "UNROLL", "LDS", "VEC", "FMA", "TWO")
PROGRAMS = ("all-pairs n-body", "gathered neighbours")


@dataclass
class RealBatch:
    counters: np.ndarray     # [N, E] float32, counts + 1
    cycles: np.ndarray       # [N] float32, GPU busy cycles
    nopts: np.ndarray        # [K] = 6
    opt_ids: np.ndarray      # [6 K] = 0..5 per kernel
    opt_off: np.ndarray
    row_off: np.ndarray
    sweeps: list             # (program, input, run) of each kernel
    E: int
    names: tuple

    @property
    def K(self):
        return len(self.nopts)

    @property
    def N(self):
        return int(self.row_off[-1])


def load(path: str = PATH) -> dict:
    with np.load(path, allow_pickle=False) as d:
        return {k: d[k] for k in d.files}


def batch(data: dict, sweeps) -> RealBatch:
    """The kernels (program, input, run) listed, in that order."""
    rows = []
    for p, i, r in sweeps:
        sel = np.flatnonzero((data["program"] == p) & (data["input"] == i) & (data["run"] == r))
        sel = sel[np.argsort(data["version"][sel], kind="stable")]
        if len(sel) != 64:
            raise ValueError(f"sweep {(p, i, r)} has {len(sel)} versions")
        rows.append(sel)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    K = len(sweeps)
    return RealBatch(counters=(data["counters"][rows] + 1.0).astype(np.float32),
                     cycles=data["cycles"][rows].astype(np.float32),
                     nopts=np.full(K, 6, np.int32), opt_ids=np.tile(np.arange(6, dtype=np.int32), K),
                     opt_off=(np.arange(K + 1) * 6).astype(np.int64), row_off=(np.arange(K + 1) * 64).astype(np.int64),
                     sweeps=list(sweeps), E=int(data["counters"].shape[1]), names=tuple(data["names"]))


def sweeps(program=None, inputs=(0, 1, 2), runs=(0, 1, 2)):
    progs = (0, 1) if program is None else (program,)
    return [(p, i, r) for p in progs for i in inputs for r in runs]
