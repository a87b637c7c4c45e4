"""The C-ABI library loads and exports every function include/arsel.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "arsel.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(arsel_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("arsel_create", "arsel_destroy", "arsel_select", "arsel_select_ragged",
              "arsel_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1404_0027_amd import arsel

    lib = ctypes.CDLL(arsel.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_strerror_is_host_only():
    from paper_1404_0027_amd import arsel

    lib = arsel.lib()
    assert lib.arsel_strerror(0) == b"ok"
    assert b"leading dimension" in lib.arsel_strerror(-4)
