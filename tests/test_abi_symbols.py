"""The C-ABI library loads on a machine without a GPU and exports every
function that include/miloc.h declares; the Python binding declares exactly
those functions.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "miloc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(miloc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("miloc_create", "miloc_destroy", "miloc_load_molecule", "miloc_load_model_1d",
                 "miloc_load_model_3d", "miloc_run", "miloc_get_populations", "miloc_get_spectra"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2009_12609_amd as miloc
    if not os.path.exists(miloc.LIB_PATH):
        pytest.fail("libmiloc.so not built (run python paper_2009_12609_amd/build.py)")
    lib = ctypes.CDLL(miloc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_matches_header():
    import paper_2009_12609_amd as miloc
    assert sorted(miloc.SIGNATURES) == declared_functions()


def test_version_string():
    import paper_2009_12609_amd as miloc
    assert "gfx950" in miloc.version()


def test_header_compiles_as_c():
    import subprocess
    import tempfile
    src = '#include "miloc.h"\nint main(void){ miloc_ctx* c = 0; (void)c; return (int)MILOC_OK; }\n'
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "t.c")
        open(p, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                               "-c", p, "-o", os.path.join(d, "t.o")])
