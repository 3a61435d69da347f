"""The C-ABI library loads (no GPU needed) and exports every function include/*.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1111_0983_amd", "libghostmg.so")


def _declared():
    names = set()
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        src = re.sub(r"#[^\n]*", " ", src)
        src = re.sub(r"typedef[^;]*;", " ", src)
        src = re.sub(r"\b(enum|struct)\s+\w*\s*\{.*?\}\s*\w*\s*;", " ", src, flags=re.S)
        for m in re.finditer(r"\b([A-Za-z_]\w*)\s*\([^;{}]*\)\s*;", src):
            names.add(m.group(1))
    return names


def test_headers_declare_the_boundary():
    names = _declared()
    for must in ("mg_setup", "mg_solve", "mg_free", "mg_strerror", "cnn_wgrad"):
        assert must in names, must


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.mg_strerror.restype = ctypes.c_char_p
    assert lib.mg_strerror(0) == b"ok"
    assert lib.mg_strerror(-4) == b"unusable geometry"
