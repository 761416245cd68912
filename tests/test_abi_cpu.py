"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(cd_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["cd_build_tree", "cd_precompute_weights", "cd_column_densities", "cd_screening_factor",
              "cd_directions", "cd_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1410_0624_amd import colden
    path = colden.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libcolden.so not built")
    lib = ctypes.CDLL(path)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(colden.EXPORTS) <= _declared()
