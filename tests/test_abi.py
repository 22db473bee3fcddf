"""The C-ABI library loads and exports every entry point include/sugg.h
declares, and the Python binding declares exactly those (no compute calls:
CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_names():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"SUGG_API[^;]*?\b(sugg_\w+)\s*\(", src, re.S))
    return names


def test_header_declares_the_boundary():
    names = header_names()
    for n in ("sugg_load_features", "sugg_fit", "sugg_predict", "sugg_rank_suggest", "sugg_suggest"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1910_07776_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libsugg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for n in header_names():
        assert hasattr(lib, n), n
    assert set(_abi.SIGNATURES) == header_names()
