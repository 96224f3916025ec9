"""The C ABI without a GPU: the shared library loads, exports every function
the public header declares, the binding lists exactly those names, and the
binding's ctypes structures have the C layout (compared with a C program
built against the header)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hodlr_fde.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("typedef")))


@pytest.fixture(scope="module")
def lib_path():
    from paper_1804_05522_amd import hodlr
    p = hodlr.LIB_PATH
    if not os.path.exists(p):
        pytest.skip("library not built (run __graft_entry__.build())")
    return p


def test_header_declares_the_api():
    names = header_functions()
    assert "hodlr_build" in names and "fde2d_sylvester_step" in names
    assert len(names) >= 17


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_header(lib_path):
    from paper_1804_05522_amd import hodlr
    assert sorted(hodlr.EXPORTS) == header_functions()


def test_host_only_entry_points(lib_path):
    """Calls that do no device work: status strings and default options."""
    from paper_1804_05522_amd import hodlr
    lib = ctypes.CDLL(lib_path)
    lib.hodlr_status_string.restype = ctypes.c_char_p
    for s in range(0, 8):
        assert lib.hodlr_status_string(s)
    o = hodlr.HodlrOpts()
    assert lib.hodlr_default_opts(ctypes.byref(o)) == 0
    assert o.leaf == 64 and 0 < o.tol < 1e-6
    assert lib.hodlr_default_opts(None) != 0


STRUCTS = ["fde_operator", "hodlr_opts", "hodlr_info", "hodlr_mat_info", "lr_matrix", "fde2d_opts", "hodlr_tuning"]


def test_struct_layout_matches_c(tmp_path):
    from paper_1804_05522_amd import hodlr
    src = tmp_path / "sizes.c"
    body = "\n".join(f'  printf("{s} %zu\\n", sizeof({s}));' for s in STRUCTS)
    src.write_text(f'#include <stdio.h>\n#include "hodlr_fde.h"\nint main(void) {{\n{body}\n  return 0;\n}}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    sizes = dict(l.split() for l in out if l)
    py = {"fde_operator": hodlr.FdeOperator, "hodlr_opts": hodlr.HodlrOpts, "hodlr_info": hodlr.HodlrInfo,
          "hodlr_mat_info": hodlr.HodlrMatInfo, "lr_matrix": hodlr.LrMatrix, "fde2d_opts": hodlr.Fde2dOpts,
          "hodlr_tuning": hodlr.HodlrTuning}
    for s in STRUCTS:
        assert int(sizes[s]) == ctypes.sizeof(py[s]), s
