"""The C-ABI library builds, loads without a GPU, and exports every function
that include/gpolylla.h declares.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpolylla.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpolylla_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2403_14723_amd as gp
    if not os.path.exists(gp.LIB_PATH):
        from paper_2403_14723_amd import build_lib
        build_lib.build()
    return gp.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gpolylla_build_halfedges", "gpolylla_mesh", "gpolylla_mesh_batch",
                 "gpolylla_result_copy", "gpolylla_strerror"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_2403_14723_amd as gp
    assert sorted(gp.exported_symbols()) == declared_functions()


def test_strerror_without_gpu(lib):
    import paper_2403_14723_amd as gp
    assert "zero-area" in gp.gpolylla_strerror(gp.GP_EDEGEN)
    assert gp.gpolylla_strerror(12345) == "unknown error"


def test_argument_errors_without_gpu(lib):
    """Null arguments are rejected before any device work."""
    import paper_2403_14723_amd as gp
    assert lib.gpolylla_mesh(None, None, 0, None) == gp.GP_EINVAL
    assert lib.gpolylla_build_halfedges(None, None, 0, None, 0, 0, None) == gp.GP_EINVAL
    assert lib.gpolylla_result_info(None, None) == gp.GP_EINVAL
    assert lib.gpolylla_ctx_set_launch(None, b"label=256x4") == gp.GP_EINVAL
    assert lib.gpolylla_ctx_get_launch(None, None, 0) == gp.GP_EINVAL
