"""Persistent cache of autotuned launch shapes, keyed by device architecture
and a shape bucket of the batch (events, optimisation-count range, log2 of
the row count, dtype, suggestions per kernel)."""
from __future__ import annotations

import json
import math
import os

import numpy as np

DEFAULT_PATH = os.environ.get("SUGG_TUNE_CACHE", os.path.expanduser("~/.cache/sugg/autotune.json"))


def arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def plan_key(plan, n_suggest: int) -> str:
    b = np.asarray(plan.nopts)
    bmin, bmax = (int(b.min()), int(b.max())) if len(b) else (0, 0)
    nb = int(math.log2(max(plan.N, 1)))
    dt = "f32" if str(plan.dtype).endswith("float32") else "f64"
    return f"{arch()}|E{plan.E}|B{bmin}-{bmax}|N2^{nb}|{dt}|n{n_suggest}"


class TuneCache(dict):
    """A dict that saves itself to a JSON file on every update."""

    def __init__(self, path: str = DEFAULT_PATH):
        super().__init__()
        self.path = path
        if os.path.exists(path):
            try:
                self.update(json.load(open(path)))
            except (OSError, ValueError):
                pass

    def __setitem__(self, k, v):
        super().__setitem__(k, v)
        try:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            with open(self.path + ".tmp", "w") as f:
                json.dump(dict(self), f, indent=1)
            os.replace(self.path + ".tmp", self.path)
        except OSError:
            pass
