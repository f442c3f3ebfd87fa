"""The C-ABI library loads and exports every function include/cprmi.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1606_00548_amd", "libcprmi.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cprmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*[\s\*]+([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_three_hot_path_calls():
    names = declared_functions()
    for n in ("assemble_jacobian", "cpr_setup", "cpr_gmres_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcprmi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    src = open(os.path.join(ROOT, "paper_1606_00548_amd", "cprmi.py")).read()
    for n in declared_functions():
        assert f'"{n}"' in src, n
