"""The C-ABI library loads and exports every entry point that include/mx.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mx.h")
LIB = os.path.join(ROOT, "paper_2601_16791_amd", "libmx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mx_init_system", "mx_step", "mx_energy", "mx_encounters", "mx_destroy",
                     "mx_get_state", "mx_set_state", "mx_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmx.so not built")
def test_params_struct_layout_matches_header(tmp_path):
    """The binding's mx_params has the header's fields, sizes and offsets (the header
    compiled with the host C compiler)."""
    import subprocess
    import paper_2601_16791_amd as mx
    names = [f for f, _ in mx.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mx.h"\nint main(void){\n'
                   'printf("%zu\\n", sizeof(mx_params));\n' +
                   "".join(f'printf("%zu\\n", offsetof(mx_params, {f}));\n' for f in names) +
                   "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got[0] == ctypes.sizeof(mx.Params)
    assert got[1:] == [getattr(mx.Params, f).offset for f in names]
    text = open(HEADER).read()
    body = text[text.index("typedef struct {", text.index("mx_status;")):text.index("} mx_params;")]
    fields = re.findall(r"\b(?:double|int32_t)\s+([A-Za-z0-9_]+)\s*;", body)
    assert fields == [f for f, _ in mx.Params._fields_]


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2601_16791_amd._binding as b
    monkeypatch.setattr(b, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(RuntimeError):
        b.lib()
