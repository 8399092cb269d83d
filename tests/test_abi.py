"""The C-ABI library loads on a machine without a GPU and exports every
function that include/*.h declares (no compute calls here)."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02602_amd", "libchemgpu.so")


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("__")))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("chem_mech_load", "chem_integrate", "chem_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.chem_strerror.restype = ctypes.c_char_p
    lib.chem_strerror.argtypes = [ctypes.c_int]
    assert lib.chem_strerror(0) == b"ok"
    assert b"mechanism" in lib.chem_strerror(-5)


def test_binding_names_match_header():
    import importlib
    cg = importlib.import_module("paper_2506_02602_amd.chemgpu")
    for n in declared_functions():
        assert n in cg.exported_symbols() or hasattr(cg, n), n
