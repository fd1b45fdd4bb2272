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


def test_jobs_argument_errors_without_gpu(lib):
    import paper_2403_14723_amd as gp
    assert lib.gpolylla_mesh_jobs(None, None, 0, 0, 0) == gp.GP_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the C layout of the header's
    (size and every field offset), checked with the host compiler."""
    import subprocess
    import paper_2403_14723_amd as gp
    structs = {"gp_job": gp.gp_job, "gp_result_dev": gp.gp_result_dev, "gp_dev_counts": gp.gp_dev_counts,
               "gp_result_debug": gp.gp_result_debug}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            cname = fname if name != "gp_dev_counts" or not fname.startswith("reserved") else "reserved"
            off = f"offsetof({name}, {cname})" + ("" if cname == fname else f" + 4 * {fname[-1]}")
            lines.append(f'  printf("{name}.{fname} %zu\\n", (size_t)({off}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).split("\n") if l)
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(out[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
