"""The C-ABI library loads and exports every entry point include/hexfc.h
declares (no compute call: this runs without a GPU)."""
from __future__ import annotations

import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "hexfc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(hexfc_[a-z_0-9]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def lib():
    import paper_2009_06574_amd as hx
    if not os.path.exists(hx.LIB_PATH):
        from paper_2009_06574_amd import build
        build.build()
    return hx.load()


def test_header_declares_the_core_boundary():
    syms = declared_symbols()
    for s in ("hexfc_upload_mesh", "hexfc_build_fragment_lists", "hexfc_resolve", "hexfc_render_frame"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_2009_06574_amd as hx
    assert sorted(hx.ABI_SYMBOLS) == declared_symbols()


def test_status_strings(lib):
    lib.hexfc_status_string.restype = ct.c_char_p
    assert lib.hexfc_status_string(0) == b"ok"
    assert lib.hexfc_status_string(-4) == b"overflow"
    assert lib.hexfc_status_string(-6) == b"invalid state"


def test_null_arguments_rejected_without_device(lib):
    import paper_2009_06574_amd as hx
    assert lib.hexfc_create(0, None) == -1
    assert lib.hexfc_set_workspace(None, None, 0) == -1
    assert lib.hexfc_upload_mesh(None, None, 0, None, 0, None, None) == -1
    assert lib.hexfc_render_frame(None, None, None, None, None, None) == -1
    lib.hexfc_destroy(None)
    assert hx.STATUS[-4] == "HEXFC_EOVERFLOW"


def test_struct_layouts_match_header():
    import paper_2009_06574_amd as hx
    assert ct.sizeof(hx.CCamera) == 16 * 4 + 8
    assert ct.sizeof(hx.CHotspot) == 16
    assert ct.sizeof(hx.CStyle) == 4 * (8 + 1 + 3 + 3 + 2 + 3 + 2 + 2)


def test_header_is_plain_c(tmp_path):
    """include/hexfc.h compiles as strict C99 (the ABI carries no C++ or torch
    types), and the struct sizes a C compiler gives match the binding's."""
    import shutil
    import subprocess
    import paper_2009_06574_amd as hx
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "t.c"
    src.write_text('#include <stdio.h>\n#include "hexfc.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu\\n", sizeof(hexfc_camera), sizeof(hexfc_hotspot), '
                   'sizeof(hexfc_style), sizeof(hexfc_lod_info)); return 0; }\n')
    exe = tmp_path / "t"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert sizes == [ct.sizeof(hx.CCamera), ct.sizeof(hx.CHotspot), ct.sizeof(hx.CStyle), ct.sizeof(hx.CLodInfo)]
