"""The C-ABI library loads and exports every entry point include/slf.h declares
(no compute calls: this runs without a GPU)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(slf_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_entry_point():
    from paper_1812_06856_amd import slf

    if not os.path.exists(slf.LIB_PATH):
        pytest.fail("libslf.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(slf.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(slf.EXPORTED) == declared


def test_params_struct_layout_matches_header():
    from paper_1812_06856_amd import slf

    p = slf.default_params()
    assert p.struct_size == ctypes.sizeof(slf.slf_params)
    assert p.levels == 64 and abs(p.tssd_T - 0.04) < 1e-7 and p.kernel_step == 5 and p.term_mask == 7
    # the last field: a layout mismatch shows here first
    assert p.energy_mode == 0 and p.exact_margin == 0 and p.homography_fp64 == 1


def test_status_strings():
    from paper_1812_06856_amd import slf

    L = slf.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.slf_status_string(code).startswith(b"SLF_")
    assert L.slf_last_error(None) == b"context is NULL"
