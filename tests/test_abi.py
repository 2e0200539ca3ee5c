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


def test_ctypes_structs_match_the_header(tmp_path):
    """Every field of the binding's ctypes mirrors of pget_geometry,
    pget_lm_params and pget_lm_report sits at the offset the C compiler
    gives it, and the sizes agree (a program built from include/pget.h
    prints them)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    rocm_inc = "/opt/rocm/include"
    if gcc is None or not os.path.exists(os.path.join(rocm_inc, "hip", "hip_runtime_api.h")):
        pytest.skip("needs gcc and the HIP headers")
    from paper_2604_26745_amd import pget
    structs = {"pget_geometry": pget.Geometry, "pget_lm_params": pget.LMParams, "pget_lm_report": pget.LMReportC}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pget.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('    printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for field, _ in cls._fields_:
            lines.append('    printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, field, cname, field))
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I" + rocm_inc, "-I" + os.path.dirname(HEADER),
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


def test_short_replay_is_refused_on_the_host():
    """The library reads max_outer replay decisions: a shorter list is an
    argument error before anything reaches the C ABI."""
    import pytest
    from paper_2604_26745_amd import pget
    with pytest.raises(ValueError, match="replay"):
        pget.SolverParams(max_outer=5, replay=[1, 0, 1]).to_c()
    p, keep = pget.SolverParams(max_outer=3, replay=[1, 0, 1]).to_c()
    assert [p.replay[k] for k in range(3)] == [1, 0, 1] and keep
