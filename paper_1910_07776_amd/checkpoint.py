"""Checkpoints of every fitted model, as safetensors files (tensors plus a JSON
header; nothing in a file is executed on load).

The tool trains its models once, when it is installed or when the profile
database changes (Section 2), and reuses them for every later query; these
files carry them between processes.

* plain (the per-optimisation linear models of Tier 2): column statistics,
  weights and training counts (``sugg_model_get`` / ``sugg_model_set``);
  predictions after a load are bit-identical.
* M5P model trees (Section 3.4): every tree, its smoothed leaf models and the
  feature statistics (``sugg_m5p_export`` / ``sugg_m5p_import``);
  predictions after a load are bit-identical.
* IBK (Section 3.4): an instance-based learner's model is its training
  instances, so the checkpoint holds them (counters, cycles, kernel
  structure) and k; loading stores them again (``sugg_ibk_fit`` is
  deterministic), predictions after a load are bit-identical.
* surrogate: FP32 parameters, Adam moments and step count; training resumed
  from a checkpoint follows the uninterrupted run bit for bit.
"""
from __future__ import annotations

import ctypes as C
import json

import numpy as np
import torch
from safetensors.torch import load_file, save_file

from . import _abi as A
from .plain import Context, Plan, ibk_fit

FORMAT = "sugg-checkpoint-1"


def _save(path: str, kind: str, tensors: dict, meta: dict):
    t = {k: (torch.from_numpy(np.ascontiguousarray(v)) if isinstance(v, np.ndarray) else v.detach().cpu().contiguous())
         for k, v in tensors.items()}
    save_file(t, path, metadata={"format": FORMAT, "kind": kind, "meta": json.dumps(meta)})


def _load(path: str, kind: str):
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        md = f.metadata() or {}
    if md.get("format") != FORMAT or md.get("kind") != kind:
        raise ValueError(f"{path} is not a {kind} checkpoint ({md.get('format')}, {md.get('kind')})")
    return load_file(path), json.loads(md.get("meta", "{}"))


# ------------------------------------------------------------------- plain --
def save_plain(ctx: Context, path: str):
    m = ctx.model_get()
    _save(path, "plain", {k: m[k] for k in ("mu", "sigma", "W", "counts")}, {})


def load_plain(ctx: Context, path: str):
    t, _ = _load(path, "plain")
    ctx.model_set({k: t[k].numpy() for k in ("mu", "sigma", "W", "counts")})


# --------------------------------------------------------------------- M5P --
def m5p_export(ctx: Context) -> dict:
    lib = A.lib()
    E, D = C.c_int32(), C.c_int32()
    A.check(ctx.h, lib.sugg_m5p_shape(ctx.h, C.byref(E), C.byref(D)))
    E, D = E.value, D.value
    node_off = np.zeros(D + 1, np.int64)
    leaf_off = np.zeros(D + 1, np.int64)
    pd = lambda a: a.ctypes.data_as(A._PD)  # noqa: E731
    pi = lambda a: a.ctypes.data_as(A._PI32)  # noqa: E731
    pl = lambda a: a.ctypes.data_as(A._PI64)  # noqa: E731
    A.check(ctx.h, lib.sugg_m5p_export(ctx.h, 0, 0, pl(node_off), pl(leaf_off), None, None, None, None, None, None,
                                       None, None, None))
    n, nl = int(node_off[-1]), int(leaf_off[-1])
    out = {"node_off": node_off, "leaf_off": leaf_off, "feat": np.zeros(n, np.int32), "thr": np.zeros(n),
           "left": np.zeros(n, np.int32), "right": np.zeros(n, np.int32), "leaf": np.zeros(n, np.int32),
           "count": np.zeros(n, np.int64), "lw": np.zeros((nl, E + 1)), "mu": np.zeros(E), "isg": np.zeros(E)}
    A.check(ctx.h, lib.sugg_m5p_export(ctx.h, n, nl, pl(node_off), pl(leaf_off), pi(out["feat"]), pd(out["thr"]),
                                       pi(out["left"]), pi(out["right"]), pi(out["leaf"]), pl(out["count"]),
                                       pd(out["lw"]), pd(out["mu"]), pd(out["isg"])))
    return out


def m5p_import(ctx: Context, m: dict):
    c = {k: np.ascontiguousarray(v) for k, v in m.items()}
    E, D = len(c["mu"]), len(c["node_off"]) - 1
    pd = lambda a: np.ascontiguousarray(a, np.float64).ctypes.data_as(A._PD)  # noqa: E731
    pi = lambda a: np.ascontiguousarray(a, np.int32).ctypes.data_as(A._PI32)  # noqa: E731
    pl = lambda a: np.ascontiguousarray(a, np.int64).ctypes.data_as(A._PI64)  # noqa: E731
    keep = [np.ascontiguousarray(c[k]) for k in c]   # the arrays outlive the call
    A.check(ctx.h, A.lib().sugg_m5p_import(ctx.h, E, D, pl(c["node_off"]), pl(c["leaf_off"]), pi(c["feat"]),
                                           pd(c["thr"]), pi(c["left"]), pi(c["right"]), pi(c["leaf"]),
                                           pl(c["count"]), pd(c["lw"]), pd(c["mu"]), pd(c["isg"])))
    del keep


def save_m5p(ctx: Context, path: str):
    _save(path, "m5p", m5p_export(ctx), {})


def load_m5p(ctx: Context, path: str):
    t, _ = _load(path, "m5p")
    m5p_import(ctx, {k: v.numpy() for k, v in t.items()})


# --------------------------------------------------------------------- IBK --
def save_ibk(path: str, plan: Plan, counters: torch.Tensor, cycles: torch.Tensor, k: int = 10):
    """The IBK model of ``ibk_fit(ctx, plan, counters, cycles, k)``: its
    training instances and k."""
    _save(path, "ibk", {"nopts": plan.nopts, "opt_ids": plan.opt_ids, "counters": counters, "cycles": cycles},
          {"E": plan.E, "D": plan.D, "k": int(k)})


def load_ibk(ctx: Context, path: str) -> Plan:
    """Stores the checkpoint's instances as the context's IBK model; returns
    the training plan (keep it alive while the model is used)."""
    t, meta = _load(path, "ibk")
    plan = Plan(ctx, t["nopts"].numpy(), t["opt_ids"].numpy(), meta["E"], meta["D"], dtype=t["counters"].dtype)
    c, cy = t["counters"].to(ctx.device), t["cycles"].to(ctx.device)
    ibk_fit(ctx, plan, c, cy, meta["k"])
    return plan


# --------------------------------------------------------------- surrogate --
def save_surrogate(mlp, path: str):
    sd = mlp.state_dict()
    _save(path, "surrogate", {"params": sd["params"], "m": sd["m"], "v": sd["v"]},
          {"shape": list(sd["shape"]), "step": int(sd["step"]), "max_batch": int(mlp.max_batch)})


def load_surrogate(ctx: Context, path: str, max_batch: int | None = None):
    """A new MLP with the checkpoint's parameters, moments and step."""
    from .surrogate import MLP
    t, meta = _load(path, "surrogate")
    i, h, o = meta["shape"]
    mlp = MLP(ctx, i, h, o, max_batch=max_batch or meta["max_batch"], params=t["params"].numpy())
    mlp.load_state_dict({"params": t["params"].to(ctx.device), "m": t["m"].to(ctx.device),
                         "v": t["v"].to(ctx.device), "step": meta["step"], "shape": (i, h, o)})
    return mlp
