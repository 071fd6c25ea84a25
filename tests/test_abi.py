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
def test_params_struct_layout_matches_header():
    import paper_2601_16791_amd as mx
    # 5 doubles, 4 int32, 10 doubles
    assert ctypes.sizeof(mx.Params) == 5 * 8 + 4 * 4 + 10 * 8
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
