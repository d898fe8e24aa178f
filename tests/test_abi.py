"""The C-ABI library loads and exports every symbol its header declares (CPU, no compute calls)."""
import ctypes
import os
import re

from paper_2101_08053_amd import igatrim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(igatrim.LIB_PATH):
        from paper_2101_08053_amd import build
        build.build(verbose=False)


def test_exports_match_header():
    _ensure_built()
    hdr = open(os.path.join(ROOT, "include", "iga_trim.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(iga_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations found"
    L = ctypes.CDLL(igatrim.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(igatrim.EXPORTED)


def test_status_strings():
    _ensure_built()
    L = ctypes.CDLL(igatrim.LIB_PATH)
    L.iga_status_string.restype = ctypes.c_char_p
    assert L.iga_status_string(0) == b"ok"
    assert L.iga_status_string(-5) == b"singular weight system"
