"""ctypes declarations of libsugg.so (the C ABI in include/sugg.h).

The library is loaded from this package's ``_lib`` folder; there is no
fallback: if it is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libsugg.so")

SUGG_OK = 0
ERRORS = {
    -1: "SUGG_E_ARG", -2: "SUGG_E_SHAPE", -3: "SUGG_E_BAD_COUNTER", -4: "SUGG_E_UNTRAINED_OPT",
    -5: "SUGG_E_SINGULAR", -6: "SUGG_E_BUDGET", -7: "SUGG_E_HIP", -8: "SUGG_E_STATE",
}
SUGG_F32, SUGG_F64 = 0, 1
SUGG_FIT_STATS, SUGG_APPLY, SUGG_BASELINE = 1, 2, 4
SUGG_MAX_OPTS = 12
SUGG_MAX_EVENTS = 256
SUGG_MAX_GLOBAL_OPTS = 64
SUGG_MAX_SUGGEST = 8
SUGG_TUNE_CANDIDATES = 61


class SuggError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Params(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("tau", C.c_double),
                ("n_suggest", C.c_int32), ("reserved", C.c_int32)]


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_PI32 = C.POINTER(C.c_int32)
_PI64 = C.POINTER(C.c_int64)
_PD = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "sugg_create": (_I32, [C.POINTER(_P), _I32, C.POINTER(Params)]),
    "sugg_destroy": (None, [_P]),
    "sugg_last_error": (C.c_char_p, [_P]),
    "sugg_set_params": (_I32, [_P, C.POINTER(Params)]),
    "sugg_get_params": (_I32, [_P, C.POINTER(Params)]),
    "sugg_plan_create": (_I32, [_P, _I32, _I32, _I32, _I32, _PI32, _PI32, C.POINTER(_P)]),
    "sugg_plan_destroy": (None, [_P]),
    "sugg_plan_rows": (_I64, [_P]),
    "sugg_plan_max_opts": (_I32, [_P]),
    "sugg_plan_set_launch": (_I32, [_P, _I32, _I32, _I32]),
    "sugg_plan_get_launch": (_I32, [_P, _PI32, _PI32, _PI32]),
    "sugg_autotune": (_I32, [_P, _P, _P, _P, _I32, C.POINTER(C.c_float), _I32, _P]),
    "sugg_plan_set_items": (_I32, [_P, _P, _I32]),
    "sugg_plan_get_items": (_I32, [_P]),
    "sugg_load_features": (_I32, [_P, _P, _P, _P, _I32, _P, _P]),
    "sugg_load_features_noalloc": (_I32, [_P, _P, _P, _P, _I32, _P, _P]),
    "sugg_fit": (_I32, [_P, _P, _P, _P, _P]),
    "sugg_predict": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "sugg_rank_suggest": (_I32, [_P, _I32, _P, _P, _I32, _I32, _I32, C.c_double, _P, _P, _P, _P]),
    "sugg_suggest": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_sync": (_I32, [_P, _P]),
    "sugg_suggest_subset": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_judge": (_I32, [_P, _P, _P, _P, _P, _I32, _P, _P, C.c_double, _P, _I32, _P]),
    "sugg_band_select": (_I32, [_P, _I32, _P, _P, _I32, _I32, _P, _P, _I32, C.c_double, C.c_double, _I32, _P,
                                _P, _P, _P]),
    "sugg_mlp_launch_info": (_I32, [_P, _PI32]),
    "sugg_mlp_freeze": (_I32, [_P, _P, _P, _P]),
    "sugg_serve_query": (_I32, [_P, _P, _P, _P, _P, C.c_double, C.c_double, _I32, _P, _P, _P, _P, _P]),
    "sugg_predict_allpaths": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_greedy": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_ibk_fit": (_I32, [_P, _P, _P, _P, _I32, _P]),
    "sugg_ibk_counts": (_I32, [_P, _P, _I32]),
    "sugg_ibk_exact_count": (_I32, [_P, _P, _PI64]),
    "sugg_ibk_predict": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "sugg_ibk_suggest": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_m5p_fit": (_I32, [_P, _P, _P, _P, _I32, C.c_double, _P]),
    "sugg_m5p_tree": (_I32, [_P, _I32, _I32, _P, _P, _P, _P, _P, _PI32]),
    "sugg_m5p_predict": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "sugg_m5p_suggest": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_m5p_shape": (_I32, [_P, _PI32, _PI32]),
    "sugg_m5p_export": (_I32, [_P, _I64, _I64, _PI64, _PI64, _PI32, _PD, _PI32, _PI32, _PI32, _PI64, _PD, _PD, _PD]),
    "sugg_m5p_import": (_I32, [_P, _I32, _I32, _PI64, _PI64, _PI32, _PD, _PI32, _PI32, _PI32, _PI64, _PD, _PD, _PD]),
    "sugg_capture_begin": (_I32, [_P, _P]),
    "sugg_capture_end": (_I32, [_P, _P, C.POINTER(_P)]),
    "sugg_graph_launch": (_I32, [_P, _P, _P]),
    "sugg_graph_destroy": (None, [_P]),
    "sugg_mlp_create": (_I32, [_P, _I32, _I32, _I32, _I32, C.POINTER(_P)]),
    "sugg_mlp_destroy": (None, [_P]),
    "sugg_mlp_param_count": (_I64, [_P]),
    "sugg_mlp_forward": (_I32, [_P, _P, _P, _P, _I32, _P, _I32, _P]),
    "sugg_mlp_loss": (_I32, [_P, _P, _P, _P, _P, _I32, _P, _P, _P]),
    "sugg_mlp_backward": (_I32, [_P, _P, _P, _P, _I32, _P, _P]),
    "sugg_mlp_adam": (_I32, [_P, _P, _P, _P, _P, _P, _I32, C.c_float, C.c_float, C.c_float, C.c_float, _P]),
    "sugg_mlp_train_step": (_I32, [_P, _P, _P, _P, _P, _P, _I32, C.c_float, _P, _P, _I32, _P, _P]),
    "sugg_surrogate_suggest": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sugg_mlp_infer": (_I32, [_P, _P, _P, _I32, _P, _P]),
    "sugg_mlp_infer_rank": (_I32, [_P, _P, _P, _I32, _I32, _I32, C.c_float, _P, _P, _P, _P, _P]),
    "sugg_mlp_train_epoch": (_I32, [_P, _P, _P, _P, _P, _P, _I32, C.c_float, _P, _P, _I64, _P, _I32, _I32, _P,
                                    _P]),
    "sugg_model_shape": (_I32, [_P, _PI32, _PI32]),
    "sugg_model_get": (_I32, [_P, _PD, _PD, _PD, _PI64]),
    "sugg_model_set": (_I32, [_P, _I32, _I32, _PD, _PD, _PD, _PI64]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1910_07776_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(ctx, code: int):
    if code != SUGG_OK:
        msg = lib().sugg_last_error(ctx).decode() if ctx else ""
        raise SuggError(code, msg)
