"""CPU checks of the C-ABI library: it loads and exports every declared entry point."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "spx.h")
LIB = os.path.join(ROOT, "paper_1109_3739_amd", "libspx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("spx_spgemm_plan", "spx_spgemm_exec", "spx_spref_plan", "spx_spasgn_plan", "spx_csc_to_dcsc"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    lib.spx_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.spx_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspx.so not built")
def test_binding_lists_every_export():
    import paper_1109_3739_amd as spx
    assert set(declared_functions()) <= set(spx.EXPORTS) | {"spx_last_error", "spx_version"}


def test_oracle_shares_no_code_with_the_library():
    """The oracle and the HIP path import / include nothing of each other."""
    pkg = os.path.join(ROOT, "paper_1109_3739_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.findall(r"^\s*(?:import|from|#include)\s+\S*", src, flags=re.M).__str__()
    osrc = open(os.path.join(ROOT, "oracle", "oracle.cpp")).read() + open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert not re.search(r"^\s*(import|from)\s+paper_1109_3739_amd", osrc, flags=re.M)
    assert not re.search(r"#include\s+[\"<]spx", osrc)
