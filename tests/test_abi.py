"""The C-ABI library loads and exports every entry point include/ipmg.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipmg.h")
LIB = os.path.join(ROOT, "paper_1606_06201_amd", "libipmg.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipmg_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("ipmg_create", "ipmg_apply_K", "ipmg_vcycle", "ipmg_pcg", "ipmg_ip_step",
                 "ipmg_element_sens", "ipmg_pcg_noalloc"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libipmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1606_06201_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared())
