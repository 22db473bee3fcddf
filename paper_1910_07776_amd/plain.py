"""Python binding of the plain scoring path (argument marshalling only).

Every function passes torch tensors' device pointers and torch's current HIP
stream to libsugg; all arithmetic runs in the library's HIP kernels.

    ctx  = Context(device=0)
    plan = Plan(ctx, nopts, opt_ids, E=128, D=6)          # host structure
    fit(ctx, train_plan, train_counters, train_cycles)    # Tier 2 training
    idx, score, count, table = suggest(ctx, plan, counters, cycles)
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _abi as A

TAU = math.log(1.05)
_DT = {torch.float32: A.SUGG_F32, torch.float64: A.SUGG_F64}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """A library context: fitted model, parameters, device status word."""

    def __init__(self, device: int = 0, lam: float = 1e-2, tau: float = TAU, n_suggest: int = 3):
        L = A.lib()
        h = C.c_void_p()
        p = A.Params(lam, tau, n_suggest, 0)
        A.check(None, L.sugg_create(C.byref(h), int(device), C.byref(p)))
        self.h = h
        self.device = torch.device("cuda", int(device))

    def close(self):
        if getattr(self, "h", None):
            A.lib().sugg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self):
        p = A.Params()
        A.check(self.h, A.lib().sugg_get_params(self.h, C.byref(p)))
        return {"lam": p.lambda_, "tau": p.tau, "n_suggest": p.n_suggest}

    def set_params(self, lam=None, tau=None, n_suggest=None):
        cur = self.params
        p = A.Params(cur["lam"] if lam is None else lam, cur["tau"] if tau is None else tau,
                     cur["n_suggest"] if n_suggest is None else n_suggest, 0)
        A.check(self.h, A.lib().sugg_set_params(self.h, C.byref(p)))

    # model checkpoint
    def model_get(self):
        E, D = C.c_int32(), C.c_int32()
        A.check(self.h, A.lib().sugg_model_shape(self.h, C.byref(E), C.byref(D)))
        E, D = E.value, D.value
        mu, sg = np.zeros(E), np.zeros(E)
        W = np.zeros((D, E + 1))
        cnt = np.zeros(D, dtype=np.int64)
        f = A.lib().sugg_model_get
        A.check(self.h, f(self.h, mu.ctypes.data_as(A._PD), sg.ctypes.data_as(A._PD),
                          W.ctypes.data_as(A._PD), cnt.ctypes.data_as(A._PI64)))
        return {"mu": mu, "sigma": sg, "W": W, "counts": cnt}

    def model_set(self, m):
        mu = np.ascontiguousarray(m["mu"], dtype=np.float64)
        sg = np.ascontiguousarray(m["sigma"], dtype=np.float64)
        W = np.ascontiguousarray(np.nan_to_num(m["W"]), dtype=np.float64)
        cnt = np.ascontiguousarray(m["counts"], dtype=np.int64)
        A.check(self.h, A.lib().sugg_model_set(self.h, len(mu), W.shape[0], mu.ctypes.data_as(A._PD),
                                               sg.ctypes.data_as(A._PD), W.ctypes.data_as(A._PD),
                                               cnt.ctypes.data_as(A._PI64)))


class Plan:
    """Structure of a batch: per-kernel optimisation counts and global ids."""

    def __init__(self, ctx: Context, nopts, opt_ids, E: int, D: int, dtype=torch.float32):
        self.ctx = ctx
        self.nopts = np.ascontiguousarray(nopts, dtype=np.int32)
        self.opt_ids = np.ascontiguousarray(opt_ids, dtype=np.int32)
        self.K, self.E, self.D, self.dtype = len(self.nopts), int(E), int(D), dtype
        if dtype not in _DT:
            raise TypeError(f"unsupported dtype {dtype}")
        h = C.c_void_p()
        L = A.lib()
        A.check(ctx.h, L.sugg_plan_create(ctx.h, self.K, self.E, self.D, _DT[dtype],
                                          self.nopts.ctypes.data_as(A._PI32),
                                          self.opt_ids.ctypes.data_as(A._PI32), C.byref(h)))
        self.h = h
        self.N = int(L.sugg_plan_rows(h))
        self.Bmax = int(L.sugg_plan_max_opts(h))
        self.row_off = np.concatenate([[0], np.cumsum(np.left_shift(1, self.nopts.astype(np.int64)))])

    def close(self):
        if getattr(self, "h", None):
            A.lib().sugg_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, waves: int, unroll: int, grid: int = 0):
        A.check(self.ctx.h, A.lib().sugg_plan_set_launch(self.h, waves, unroll, grid))

    def set_items(self, rows: int):
        """Target rows of a work item of the scoring pass (rebuilds the work list)."""
        A.check(self.ctx.h, A.lib().sugg_plan_set_items(self.ctx.h, self.h, int(rows)))

    def get_items(self) -> int:
        return int(A.lib().sugg_plan_get_items(self.h))

    def get_launch(self):
        w, u, g = C.c_int32(), C.c_int32(), C.c_int32()
        A.check(self.ctx.h, A.lib().sugg_plan_get_launch(self.h, C.byref(w), C.byref(u), C.byref(g)))
        return {"waves": w.value, "unroll": u.value, "grid": g.value}

    def check_inputs(self, counters, cycles):
        for name, t, shape in (("counters", counters, (self.N, self.E)), ("cycles", cycles, (self.N,))):
            if not isinstance(t, torch.Tensor) or t.device != self.ctx.device:
                raise ValueError(f"{name} must be a tensor on {self.ctx.device}")
            if t.dtype != self.dtype or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous {self.dtype} of shape {shape}")


def load_features(ctx: Context, plan: Plan, counters, cycles, fit_stats: bool = False,
                  apply: bool = True, baseline: bool = False):
    """Tier 1 features; returns the standardised features when apply: N x E,
    or K x E of the baseline versions only when baseline."""
    plan.check_inputs(counters, cycles)
    mode = (A.SUGG_FIT_STATS if fit_stats else 0) | (A.SUGG_APPLY if apply else 0) | \
        (A.SUGG_BASELINE if baseline else 0)
    rows = plan.K if baseline else plan.N
    z = torch.empty((rows, plan.E), dtype=plan.dtype, device=ctx.device) if apply else None
    A.check(ctx.h, A.lib().sugg_load_features(ctx.h, plan.h, _ptr(counters), _ptr(cycles), mode,
                                              _ptr(z), _stream()))
    return z


def load_features_noalloc(ctx: Context, plan: Plan, counters, cycles, fit_stats: bool = False,
                          apply: bool = True, baseline: bool = False, z=None):
    """load_features through the entry point that allocates no device memory
    (statistics partials in the library's static scratch); z (optional) is a
    preallocated output, so the call itself allocates nothing."""
    plan.check_inputs(counters, cycles)
    mode = (A.SUGG_FIT_STATS if fit_stats else 0) | (A.SUGG_APPLY if apply else 0) | \
        (A.SUGG_BASELINE if baseline else 0)
    if apply and z is None:
        z = torch.empty((plan.K if baseline else plan.N, plan.E), dtype=plan.dtype, device=ctx.device)
    A.check(ctx.h, A.lib().sugg_load_features_noalloc(ctx.h, plan.h, _ptr(counters), _ptr(cycles), mode,
                                                      _ptr(z), _stream()))
    return z


def fit(ctx: Context, plan: Plan, counters, cycles):
    """Tier 2 training on every before/after pair of the plan's kernels."""
    plan.check_inputs(counters, cycles)
    A.check(ctx.h, A.lib().sugg_fit(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _stream()))


def predict(ctx: Context, plan: Plan, counters, cycles, grid: bool = False):
    """Returns (table [N], grid [N, Bmax] or None)."""
    plan.check_inputs(counters, cycles)
    table = torch.empty(plan.N, dtype=plan.dtype, device=ctx.device)
    g = torch.empty((plan.N, plan.Bmax), dtype=plan.dtype, device=ctx.device) if grid else None
    A.check(ctx.h, A.lib().sugg_predict(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(g),
                                        _ptr(table), _stream()))
    return table, g


def suggest(ctx: Context, plan: Plan, counters, cycles, table: bool = True, out=None):
    """The fused path; returns (idx [K, n], score [K, n], count [K], table [N] or None).
    ``out`` may hold preallocated tensors with the same keys."""
    plan.check_inputs(counters, cycles)
    n = ctx.params["n_suggest"]
    if out is None:
        out = {"idx": torch.empty((plan.K, n), dtype=torch.int32, device=ctx.device),
               "score": torch.empty((plan.K, n), dtype=plan.dtype, device=ctx.device),
               "count": torch.empty(plan.K, dtype=torch.int32, device=ctx.device),
               "table": torch.empty(plan.N, dtype=plan.dtype, device=ctx.device) if table else None}
    A.check(ctx.h, A.lib().sugg_suggest(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(out["table"]),
                                        _ptr(out["idx"]), _ptr(out["score"]), _ptr(out["count"]), _stream()))
    return out["idx"], out["score"], out["count"], out["table"]


def suggest_subset(ctx: Context, plan: Plan, counters, cycles, kmask, out):
    """Re-score only the kernels with kmask[k] != 0 (int32 [K] device tensor),
    writing their entries of ``out`` (as returned by ``suggest``)."""
    plan.check_inputs(counters, cycles)
    if kmask.dtype != torch.int32 or kmask.numel() != plan.K or kmask.device != ctx.device:
        raise ValueError("kmask must be an int32 tensor of K entries on the context device")
    A.check(ctx.h, A.lib().sugg_suggest_subset(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(kmask),
                                               _ptr(out["table"]), _ptr(out["idx"]), _ptr(out["score"]),
                                               _ptr(out["count"]), _stream()))
    return out


def judge(ctx: Context, plan: Plan, counters, cycles, cand, out=None, ref=None, tol: float = 0.1, flag=None,
          accumulate: bool = False):
    """Plain composed log-speedups of candidate subsets cand [K, C] (int32,
    < 0 = none), reading only each subset's chain of versions.  With ref
    (values to check, [K, C]) and flag (int32 [K]): flag[k] = 1 where some
    candidate differs from ref by more than tol (``accumulate``: flags
    already set stay set)."""
    plan.check_inputs(counters, cycles)
    if cand.dtype != torch.int32 or cand.dim() != 2 or cand.shape[0] != plan.K or not cand.is_contiguous():
        raise ValueError("cand must be a contiguous int32 [K, C] tensor")
    if out is None:
        out = torch.empty(tuple(cand.shape), dtype=plan.dtype, device=ctx.device)
    if (ref is None) != (flag is None):
        raise ValueError("ref and flag go together")
    A.check(ctx.h, A.lib().sugg_judge(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(cand), cand.shape[1],
                                      _ptr(out), _ptr(ref), float(tol), _ptr(flag), int(bool(accumulate)),
                                      _stream()))
    return out


def surrogate_suggest(ctx: Context, plan: Plan, mlp, counters, cycles, table: bool = False, out=None):
    """The frozen surrogate's top-n subsets of every kernel of a uniform
    batch in one library call (baseline features in BF16, the network,
    Tier 3 in its output layer); returns (idx, score, count, table or None)."""
    plan.check_inputs(counters, cycles)
    n = ctx.params["n_suggest"]
    K, V = plan.K, 1 << int(plan.Bmax)
    if out is None:
        out = {"idx": torch.empty((K, n), dtype=torch.int32, device=ctx.device),
               "score": torch.empty((K, n), dtype=plan.dtype, device=ctx.device),
               "count": torch.empty(K, dtype=torch.int32, device=ctx.device),
               "table": torch.empty((K, V), dtype=plan.dtype, device=ctx.device) if table else None}
    A.check(ctx.h, A.lib().sugg_surrogate_suggest(ctx.h, plan.h, mlp.h, _ptr(counters), _ptr(cycles),
                                                  _ptr(out.get("table")), _ptr(out["idx"]), _ptr(out["score"]),
                                                  _ptr(out["count"]), _stream()))
    return out["idx"], out["score"], out["count"], out.get("table")


def serve_query(ctx: Context, plan: Plan, mlp, counters, cycles, out, flag, tol: float = 0.1, band: float = 0.1,
                cap: int = 16):
    """One serving query in a single call (surrogate, top-n, threshold band,
    judge, plain fallback; see sugg_serve_query): writes out = {"idx",
    "score", "count"} and flag [K] (1 where the plain path answered)."""
    plan.check_inputs(counters, cycles)
    A.check(ctx.h, A.lib().sugg_serve_query(ctx.h, plan.h, mlp.h, _ptr(counters), _ptr(cycles), float(tol),
                                            float(band), int(cap), _ptr(out["idx"]), _ptr(out["score"]),
                                            _ptr(out["count"]), _ptr(flag), _stream()))
    return flag


def predict_allpaths(ctx: Context, plan: Plan, counters, cycles, rank: bool = True):
    """All-paths composed table [N] (the mean over every order of adding a
    subset's optimisations) and, with rank, its top-n per kernel:
    returns (table, idx, score, count) (the last three None without rank)."""
    plan.check_inputs(counters, cycles)
    n = ctx.params["n_suggest"]
    table = torch.empty(plan.N, dtype=plan.dtype, device=ctx.device)
    idx = torch.empty((plan.K, n), dtype=torch.int32, device=ctx.device) if rank else None
    sc = torch.empty((plan.K, n), dtype=plan.dtype, device=ctx.device) if rank else None
    cnt = torch.empty(plan.K, dtype=torch.int32, device=ctx.device) if rank else None
    A.check(ctx.h, A.lib().sugg_predict_allpaths(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(table),
                                                 _ptr(idx), _ptr(sc), _ptr(cnt), _stream()))
    return table, idx, sc, cnt


def greedy(ctx: Context, plan: Plan, counters, cycles):
    """Greedy re-profiling per kernel: returns (path [K, Bmax+1] int32 of the
    visited versions from 0, -1 after the last; steps [K]; gain [K], the sum
    of the predicted benefits of the steps)."""
    plan.check_inputs(counters, cycles)
    path = torch.empty((plan.K, plan.Bmax + 1), dtype=torch.int32, device=ctx.device)
    steps = torch.empty(plan.K, dtype=torch.int32, device=ctx.device)
    gain = torch.empty(plan.K, dtype=plan.dtype, device=ctx.device)
    A.check(ctx.h, A.lib().sugg_greedy(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(path), _ptr(steps),
                                       _ptr(gain), _stream()))
    return path, steps, gain


# ---- instance-based Tier 2 model (IBK) ---------------------------------------
def ibk_fit(ctx: Context, plan: Plan, counters, cycles, k: int = 10):
    """Store every before/after pair of the plan's kernels as IBK samples (k
    nearest neighbours, mean label); replaces the context's IBK model."""
    plan.check_inputs(counters, cycles)
    A.check(ctx.h, A.lib().sugg_ibk_fit(ctx.h, plan.h, _ptr(counters), _ptr(cycles), int(k), _stream()))


def ibk_counts(ctx: Context, D: int) -> np.ndarray:
    out = np.zeros(D, dtype=np.int64)
    A.check(ctx.h, A.lib().sugg_ibk_counts(ctx.h, out.ctypes.data_as(C.c_void_p), D))
    return out


def ibk_exact_count(ctx: Context, plan: Plan) -> int:
    """Queries of the plan's last IBK call whose FP32 candidates could not be
    certified and were searched again over all samples in FP64."""
    n = C.c_int64()
    A.check(ctx.h, A.lib().sugg_ibk_exact_count(ctx.h, plan.h, C.byref(n)))
    return int(n.value)


def ibk_predict(ctx: Context, plan: Plan, counters, cycles, grid: bool = False):
    """Returns (table [N], grid [N, Bmax] or None) with IBK as Tier 2."""
    plan.check_inputs(counters, cycles)
    table = torch.empty(plan.N, dtype=plan.dtype, device=ctx.device)
    g = torch.empty((plan.N, plan.Bmax), dtype=plan.dtype, device=ctx.device) if grid else None
    A.check(ctx.h, A.lib().sugg_ibk_predict(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(g), _ptr(table),
                                            _stream()))
    return table, g


def ibk_suggest(ctx: Context, plan: Plan, counters, cycles, table: bool = True, out=None):
    """``suggest`` with IBK as Tier 2; returns (idx, score, count, table or None)."""
    plan.check_inputs(counters, cycles)
    n = ctx.params["n_suggest"]
    if out is None:
        out = {"idx": torch.empty((plan.K, n), dtype=torch.int32, device=ctx.device),
               "score": torch.empty((plan.K, n), dtype=plan.dtype, device=ctx.device),
               "count": torch.empty(plan.K, dtype=torch.int32, device=ctx.device),
               "table": torch.empty(plan.N, dtype=plan.dtype, device=ctx.device) if table else None}
    A.check(ctx.h, A.lib().sugg_ibk_suggest(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(out["table"]),
                                            _ptr(out["idx"]), _ptr(out["score"]), _ptr(out["count"]), _stream()))
    return out["idx"], out["score"], out["count"], out["table"]


def m5p_fit(ctx: Context, plan: Plan, counters, cycles, min_leaf: int = 4, smooth_k: float = 15.0):
    """Induce an M5P model tree per global id from the plan's before/after
    pairs; replaces the context's M5P model.  Synchronous."""
    plan.check_inputs(counters, cycles)
    A.check(ctx.h, A.lib().sugg_m5p_fit(ctx.h, plan.h, _ptr(counters), _ptr(cycles), int(min_leaf),
                                        float(smooth_k), _stream()))


def m5p_tree(ctx: Context, opt: int) -> dict:
    """The pruned tree of global id ``opt`` in preorder: feat (-1 at a leaf),
    thr (NaN at a leaf), left, right (-1 at a leaf), count."""
    n = C.c_int32(0)
    A.check(ctx.h, A.lib().sugg_m5p_tree(ctx.h, int(opt), 0, None, None, None, None, None, C.byref(n)))
    out = {"feat": np.zeros(n.value, np.int32), "thr": np.zeros(n.value, np.float64),
           "left": np.zeros(n.value, np.int32), "right": np.zeros(n.value, np.int32),
           "count": np.zeros(n.value, np.int64)}
    vp = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    A.check(ctx.h, A.lib().sugg_m5p_tree(ctx.h, int(opt), n.value, vp(out["feat"]), vp(out["thr"]), vp(out["left"]),
                                         vp(out["right"]), vp(out["count"]), C.byref(n)))
    return out


def m5p_predict(ctx: Context, plan: Plan, counters, cycles, grid: bool = False):
    """Returns (table [N], grid [N, Bmax] or None) with M5P as Tier 2."""
    plan.check_inputs(counters, cycles)
    table = torch.empty(plan.N, dtype=plan.dtype, device=ctx.device)
    g = torch.empty((plan.N, plan.Bmax), dtype=plan.dtype, device=ctx.device) if grid else None
    A.check(ctx.h, A.lib().sugg_m5p_predict(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(g), _ptr(table),
                                            _stream()))
    return table, g


def m5p_suggest(ctx: Context, plan: Plan, counters, cycles, table: bool = True, out=None):
    """``suggest`` with M5P as Tier 2; returns (idx, score, count, table or None)."""
    plan.check_inputs(counters, cycles)
    n = ctx.params["n_suggest"]
    if out is None:
        out = {"idx": torch.empty((plan.K, n), dtype=torch.int32, device=ctx.device),
               "score": torch.empty((plan.K, n), dtype=plan.dtype, device=ctx.device),
               "count": torch.empty(plan.K, dtype=torch.int32, device=ctx.device),
               "table": torch.empty(plan.N, dtype=plan.dtype, device=ctx.device) if table else None}
    A.check(ctx.h, A.lib().sugg_m5p_suggest(ctx.h, plan.h, _ptr(counters), _ptr(cycles), _ptr(out["table"]),
                                            _ptr(out["idx"]), _ptr(out["score"]), _ptr(out["count"]), _stream()))
    return out["idx"], out["score"], out["count"], out["table"]


def rank_suggest(ctx: Context, scores, seg_off, n: int = 3, tau: float = TAU, skip_head: int = 0, out=None):
    """Tier 3 over segments scores[seg_off[i]:seg_off[i+1]]; returns (idx, score, count),
    written into ``out`` = (idx [nseg, n], score [nseg, n], count [nseg]) when given."""
    if scores.dtype not in _DT or not scores.is_contiguous() or scores.device != ctx.device:
        raise ValueError("scores must be a contiguous float32/float64 tensor on the context device")
    if seg_off.dtype != torch.int64 or not seg_off.is_contiguous() or seg_off.device != ctx.device:
        raise ValueError("seg_off must be a contiguous int64 tensor on the context device")
    nseg = seg_off.numel() - 1
    if out is None:
        out = (torch.empty((max(nseg, 0), n), dtype=torch.int32, device=ctx.device),
               torch.empty((max(nseg, 0), n), dtype=scores.dtype, device=ctx.device),
               torch.empty(max(nseg, 0), dtype=torch.int32, device=ctx.device))
    idx, sc, cnt = out
    if (idx.shape != (max(nseg, 0), n) or sc.shape != idx.shape or cnt.numel() != max(nseg, 0)
            or idx.dtype != torch.int32 or cnt.dtype != torch.int32 or sc.dtype != scores.dtype
            or not (idx.is_contiguous() and sc.is_contiguous() and cnt.is_contiguous())):
        raise ValueError("out must be contiguous (idx int32 [nseg, n], score [nseg, n], count int32 [nseg])")
    A.check(ctx.h, A.lib().sugg_rank_suggest(ctx.h, _DT[scores.dtype], _ptr(scores), _ptr(seg_off),
                                             max(nseg, 0), skip_head, n, float(tau), _ptr(idx), _ptr(sc),
                                             _ptr(cnt), _stream()))
    return idx, sc, cnt


def band_select(ctx: Context, scores, seg_off, top_idx, top_count, tau: float = TAU, band: float = 0.1,
                cap: int = 16, skip_head: int = 0, out=None):
    """Threshold band of short lists (see ``rank_suggest``): per segment whose
    list holds fewer than n entries, the other entries with score >= tau -
    band, ascending, at most ``cap``.  Returns (cand [nseg, cap] int32,
    ref [nseg, cap] scores, flag [nseg] int32: 1 = more than cap)."""
    if scores.dtype not in _DT or not scores.is_contiguous() or scores.device != ctx.device:
        raise ValueError("scores must be a contiguous float32/float64 tensor on the context device")
    if seg_off.dtype != torch.int64 or not seg_off.is_contiguous() or seg_off.device != ctx.device:
        raise ValueError("seg_off must be a contiguous int64 tensor on the context device")
    nseg = max(seg_off.numel() - 1, 0)
    if (top_idx.dtype != torch.int32 or top_idx.dim() != 2 or top_idx.shape[0] != nseg
            or not top_idx.is_contiguous() or top_count.dtype != torch.int32 or top_count.numel() != nseg):
        raise ValueError("top_idx [nseg, n] and top_count [nseg] must be contiguous int32 tensors")
    if out is None:
        out = (torch.empty((nseg, cap), dtype=torch.int32, device=ctx.device),
               torch.empty((nseg, cap), dtype=scores.dtype, device=ctx.device),
               torch.empty(nseg, dtype=torch.int32, device=ctx.device))
    cand, ref, flag = out
    A.check(ctx.h, A.lib().sugg_band_select(ctx.h, _DT[scores.dtype], _ptr(scores), _ptr(seg_off), nseg, skip_head,
                                            _ptr(top_idx), _ptr(top_count), top_idx.shape[1], float(tau),
                                            float(band), cap, _ptr(cand), _ptr(ref), _ptr(flag), _stream()))
    return cand, ref, flag


TUNE_ITEMS = (64, 128, 256, 512, 1024)
TUNE_WAVES = (2, 4, 8)
TUNE_UNROLL = (1, 2, 4)


def autotune(ctx: Context, plan: Plan, counters, cycles, reps: int = 5, cache=None):
    """Time every launch shape of the plan's scoring kernel on these inputs
    (item size x waves x unroll, and the split form where there is one) and
    keep the fastest.  ``cache`` (a tuning.TuneCache) is consulted first and
    updated afterwards.  Returns the chosen shape and the timings."""
    from . import tuning
    key = tuning.plan_key(plan, ctx.params["n_suggest"])
    if cache is not None and key in cache:
        cfg = cache[key]
        if "items" in cfg:
            plan.set_items(cfg["items"])
        plan.set_launch(cfg["waves"], cfg["unroll"], 0)
        return cfg
    plan.check_inputs(counters, cycles)
    times = (C.c_float * A.SUGG_TUNE_CANDIDATES)()
    A.check(ctx.h, A.lib().sugg_autotune(ctx.h, plan.h, _ptr(counters), _ptr(cycles), int(reps), times,
                                         A.SUGG_TUNE_CANDIDATES, _stream()))
    cfg = plan.get_launch()
    cfg["items"] = plan.get_items()
    shapes = [f"w{w}u{u}" for w in TUNE_WAVES for u in TUNE_UNROLL] + [f"stream{u}" for u in (1, 2, 4)]
    names = [f"i{ir}{sh}" for ir in TUNE_ITEMS for sh in shapes]
    cfg["times_ms"] = {n: float(times[i]) for i, n in enumerate(names) if times[i] >= 0}
    if times[len(names)] >= 0:
        cfg["times_ms"]["split"] = float(times[len(names)])
    if cache is not None:
        cache[key] = cfg
    return cfg


class Graph:
    """Scoring passes recorded once and replayed (hipGraph).

        g = Graph(ctx)
        with g.capture():
            suggest(ctx, plan, counters, cycles, out=bufs)   # recorded, not run
        g.launch()                                           # replays in place
    """

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.h = None
        self.stream = torch.cuda.Stream(device=ctx.device)

    class _Cap:
        def __init__(self, g):
            self.g = g

        def __enter__(self):
            g = self.g
            g.stream.wait_stream(torch.cuda.current_stream(g.ctx.device))
            self.sctx = torch.cuda.stream(g.stream)
            self.sctx.__enter__()
            A.check(g.ctx.h, A.lib().sugg_capture_begin(g.ctx.h, C.c_void_p(g.stream.cuda_stream)))
            return g

        def __exit__(self, et, ev, tb):
            g = self.g
            h = C.c_void_p()
            rc = A.lib().sugg_capture_end(g.ctx.h, C.c_void_p(g.stream.cuda_stream), C.byref(h))
            self.sctx.__exit__(et, ev, tb)
            if et is None:
                A.check(g.ctx.h, rc)
                g.h = h
            return False

    def capture(self):
        if self.h is not None:
            raise RuntimeError("graph already captured")
        return Graph._Cap(self)

    def launch(self):
        A.check(self.ctx.h, A.lib().sugg_graph_launch(self.ctx.h, self.h, _stream()))

    def close(self):
        if self.h is not None:
            A.lib().sugg_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sync(ctx: Context):
    """Wait for the current stream and raise any device-detected data error."""
    A.check(ctx.h, A.lib().sugg_sync(ctx.h, _stream()))
