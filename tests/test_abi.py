"""The C ABI library loads and exports every function include/gs.h
declares, and the Python binding knows each of them.  No GPU work."""
import ctypes as C
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|size_t|double|char|float)\s*\*?\s*(gs_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    import paper_2507_23006_amd as gs
    from paper_2507_23006_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        gs.build()
    names = declared_functions()
    assert len(names) >= 20, names
    lib = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)
    loaded = _lib.load()
    assert loaded.gs_version().decode().startswith("gsmi")
