"""The C-ABI library loads and exports every symbol include/fa2lay.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fa2lay.h")
LIB = os.path.join(ROOT, "paper_2403_03504_amd", "libfa2lay.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("fl_create", "fl_build_csr", "fl_components", "fl_fa2_forces", "fl_fa2_step", "fl_fa2_run",
                 "fl_morton", "fl_tree"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libfa2lay.so is not built (run python -m paper_2403_03504_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.fl_version.restype = ctypes.c_char_p
    assert lib.fl_version().decode().startswith("fa2lay")


def test_binding_names_match_header():
    src = open(os.path.join(ROOT, "paper_2403_03504_amd", "fa2lay.py")).read()
    exported = re.search(r"EXPORTED = \((.*?)\)", src, re.S).group(1)
    names = sorted(re.findall(r'"(fl_[a-z0-9_]+)"', exported))
    assert names == declared()
