"""CPU-side checks of the C-ABI library: it loads without a GPU and exports
every entry point include/llg.h declares; the binding wraps each of them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llg.h")
LIB = os.path.join(ROOT, "paper_1102_3069_amd", "libllg.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(llg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("llg_create", "llg_set_geometry", "llg_set_cellsize", "llg_set_material",
              "llg_set_anisotropy_uniaxial", "llg_set_applied_field", "llg_set_temperature",
              "llg_set_m", "llg_eval_heff", "llg_step", "llg_run"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing


def test_binding_covers_every_declared_symbol():
    import paper_1102_3069_amd as llg
    assert sorted(llg.EXPORTS) == declared()
