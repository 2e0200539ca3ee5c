"""The C-ABI library loads and exports every entry point include/pget.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pget.h")
LIB = os.path.join(ROOT, "paper_2604_26745_amd", "libpget.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(pget_[a-z_0-9]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pget_forward", "pget_jvp", "pget_vjp", "pget_lm_solve", "pget_lm_solve_batched",
                 "pget_plan_create", "pget_plan_destroy", "pget_workspace_bytes",
                 "pget_status_string"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpget.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpget.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.pget_status_string.restype = ctypes.c_char_p
    lib.pget_status_string.argtypes = [ctypes.c_int]
    assert lib.pget_status_string(0) == b"ok"
    assert lib.pget_status_string(-1) == b"invalid argument"
    # invalid arguments are rejected before any device work
    lib.pget_plan_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.pget_plan_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.pget_plan_create(None, 0, ctypes.byref(out)) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2604_26745_amd import pget
    monkeypatch.setattr(pget, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pget, "_lib", None)
    with pytest.raises(RuntimeError):
        pget.load_library()
