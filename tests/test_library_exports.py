"""The C-ABI library loads on a machine without a GPU and exports every
function that include/foap4.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "foap4.h")
LIB = os.path.join(ROOT, "paper_2605_07612_amd", "libfoap4.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(foap4_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_paper_operations():
    names = declared()
    for n in ("foap4_mesh_create", "foap4_ghost_pattern_build", "foap4_ghost_fill", "foap4_step",
              "foap4_regrid", "foap4_batch_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfoap4.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfoap4.so not built")
def test_binding_covers_the_header():
    import paper_2605_07612_amd as f4
    assert set(declared()) <= set(f4.EXPORTS)
