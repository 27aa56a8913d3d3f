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


STRUCTS = {"gs_camera": "GsCamera", "gs_options": "GsOptions", "gs_gaussians": "GsGaussians",
           "gs_gaussians_grad": "GsGaussiansGrad", "gs_projected": "GsProjected",
           "gs_appearance_mlp": "GsAppearanceMlp", "gs_appearance_grad": "GsAppearanceGrad",
           "gs_densify_params": "GsDensifyParams", "gs_lod_table": "GsLodTable",
           "gs_serve_config": "GsServeConfig", "gs_completion": "GsCompletion", "gs_serve_stats": "GsServeStats"}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every struct of include/gs.h has the binding's size and field offsets,
    as the host C compiler lays it out."""
    import shutil
    import subprocess
    from paper_2507_23006_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    assert cc, "no host C compiler"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gs.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(_lib, pyname)
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    (tmp_path / "layout.c").write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(tmp_path / "layout.c"), "-o", str(exe)],
                   check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                             text=True).stdout.splitlines())
    for cname, pyname in STRUCTS.items():
        cls = getattr(_lib, pyname)
        assert int(got[f"{cname} size"]) == C.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(got[f"{cname}.{field}"]) == getattr(cls, field).offset, f"{cname}.{field}"
