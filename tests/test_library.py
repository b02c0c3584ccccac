"""Host-side checks of the C-ABI library (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_20536_amd", "libgxyhotrg.so")
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ \*]*?\b(gxy_[a-z0-9_]+)\s*\(",
                             txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_headers_declare_the_api():
    names = declared_symbols()
    for n in ["gxy_create", "gxy_destroy", "gxy_run", "gxy_run_batch", "gxy_char_coeffs",
              "gxy_initial_tensor", "gxy_step_log", "gxy_observables", "gxy_workspace_bytes",
              "gxy_set_workspace", "gxy_status_string", "gxy_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared_symbols()) if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_null_arguments():
    lib = ctypes.CDLL(LIB)
    lib.gxy_status_string.restype = ctypes.c_char_p
    assert lib.gxy_status_string(0) == b"ok"
    assert lib.gxy_status_string(4) == b"numerical failure"
    # every entry point rejects null handles without touching a device
    assert lib.gxy_run(None, None, None) == 1
    assert lib.gxy_run_batch(None, None, 0, None) == 1
    assert lib.gxy_destroy(None) == 1
    assert lib.gxy_create(None, 0, None) == 1


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2609_20536_amd import hotrg
    with pytest.raises(RuntimeError):
        hotrg._lib = None
        hotrg.load_library(str(tmp_path / "missing.so"))
    hotrg._lib = None


@pytest.mark.skipif(__import__("shutil").which("gcc") is None, reason="gcc not available")
def test_binding_structs_match_the_header_layout(tmp_path):
    """Size and every field offset of gxy_point, gxy_result and
    gxy_step_info as a C compiler lays them out from the header, against the
    ctypes structures of the binding."""
    import subprocess
    from paper_2609_20536_amd import hotrg as H
    structs = {"gxy_point": H.Point, "gxy_result": H.Result, "gxy_step_info": H.StepInfo,
               "gxy_lgt_result": H.LgtResult}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "gxy_hotrg.h"',
           '#include "gxy_lgt.h"', "int main(void) {"]
    for cname, cls in structs.items():
        src.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            src.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o",
                        str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
