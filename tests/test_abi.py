"""Host-side checks of the C-ABI library: it was built for gfx950, it loads,
and it exports every function include/ff.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ff.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ff_[a-z_]+)\s*\(", src)
    return [n for n in dict.fromkeys(names)]


@pytest.fixture(scope="module")
def libff():
    from paper_1805_03517_amd import ff
    if not os.path.exists(ff.LIB_PATH):
        from paper_1805_03517_amd import build
        build.build()
    return ff


def test_header_declares_the_boundary():
    decl = _declared_functions()
    for name in ("ff_create", "ff_match_pair", "ff_match_batch", "ff_destroy"):
        assert name in decl


def test_library_exports_every_declared_symbol(libff):
    lib = ctypes.CDLL(libff.LIB_PATH)
    decl = _declared_functions()
    missing = [n for n in decl if not hasattr(lib, n)]
    assert not missing, missing
    assert set(decl) == set(libff.EXPORTS)


def test_exports_are_extern_c(libff):
    out = subprocess.check_output(["nm", "-D", "--defined-only", libff.LIB_PATH], text=True)
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in _declared_functions():
        assert n in syms, n


def test_library_holds_gfx950_code_object(libff):
    data = open(libff.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_null_handle_paths_do_not_touch_the_device(libff):
    lib = libff.lib()
    assert lib.ff_last_error(None) is not None
    assert lib.ff_match_pair(None, None, None) == libff.FF_ERR_INVALID
    assert lib.ff_match_batch(None, None, 1, None) == libff.FF_ERR_INVALID
    lib.ff_destroy(None)
    assert lib.ff_workspace_bytes(None, None, 0) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1805_03517_amd import ff
    monkeypatch.setattr(ff, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ff, "_lib", None)
    with pytest.raises(ff.FFError):
        ff.lib()


def test_struct_layouts_match_the_binding(libff, tmp_path):
    """The ctypes mirrors of ff_params and ff_pair have the C layout: field
    offsets and sizes as gcc lays out include/ff.h."""
    structs = {"ff_params": libff.Params, "ff_pair": libff.Pair}
    src = ["#include <stddef.h>", "#include <stdio.h>", '#include "ff.h"', "int main(void) {"]
    for cname, py in structs.items():
        src.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            src.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src += ["return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
