"""The built library loads on the host and exports every entry point the header declares."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helmdd.h")
LIB = os.path.join(ROOT, "paper_2512_12538_amd", "libhelmdd.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = _declared()
    for n in ("hh_setup", "hh_build_coarse", "hh_solve", "hh_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (same HIP runtime as the binding)

    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_imports_and_rejects_bad_shapes_on_host():
    import paper_2512_12538_amd as hh

    hh.load()
    d = hh.decomposition([(4, 4)], [4])
    assert d.levels == 1 and d.m[0][0] == 4 and d.overlap_cells[0] == 4
    assert hh.library_path() == LIB
