"""The C-ABI library loads and exports every entry point include/lmmew.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(lmmew_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_entry_point():
    from paper_2305_17111_amd import build as libbuild

    path = libbuild.LIB
    if not os.path.exists(path):
        libbuild.build()
    lib = ctypes.CDLL(path)
    names = _declared()
    assert len(names) >= 12, names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_device():
    from paper_2305_17111_amd import build as libbuild

    lib = ctypes.CDLL(libbuild.LIB)
    lib.lmmew_status_string.restype = ctypes.c_char_p
    assert lib.lmmew_status_string(0) == b"ok"
    assert lib.lmmew_status_string(-1) == b"invalid argument"
    # NULL arguments are rejected before any device work
    assert lib.lmmew_create(None, None, None, None, None) == -1
    assert lib.lmmew_destroy(None) == -1
