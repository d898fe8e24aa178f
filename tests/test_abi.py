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


def test_index_check_count_is_a_test_build_call():
    """A release build answers IGA_E_UNSUPPORTED; the index-checking build exports the same symbols."""
    _ensure_built()
    L = ctypes.CDLL(igatrim.LIB_PATH)
    n = ctypes.c_int64(-1)
    assert L.iga_debug_bounds_hits(ctypes.byref(n), 0) == -2 and n.value == 0
    dbg = os.path.join(os.path.dirname(igatrim.LIB_PATH), "libigatrim_debug.so")
    if os.path.exists(dbg):
        hdr = open(os.path.join(ROOT, "include", "iga_trim.h")).read()
        declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(iga_\w+)\s*\(", hdr, re.M))
        D = ctypes.CDLL(dbg)
        for name in declared:
            assert hasattr(D, name), name
