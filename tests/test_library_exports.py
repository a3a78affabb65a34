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


def test_descriptor_layout_matches_the_header(tmp_path):
    """The binding's MeshDesc has the size and field offsets that a C
    compiler gives foap4_mesh_desc from include/foap4.h."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    import paper_2605_07612_amd as f4
    fields = [name for name, _ in f4.MeshDesc._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"foap4.h\"\nint main(void) {\n"
                   + "  printf(\"%zu\\n\", sizeof(foap4_mesh_desc));\n"
                   + "".join(f"  printf(\"%zu\\n\", offsetof(foap4_mesh_desc, {n}));\n" for n in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got[0] == ctypes.sizeof(f4.MeshDesc)
    assert got[1:] == [getattr(f4.MeshDesc, n).offset for n in fields]
