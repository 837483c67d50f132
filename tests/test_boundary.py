"""The C-ABI library builds for gfx950, loads, and exports every entry point that
include/lpdec.h declares (no compute: there is no GPU on the build host)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "lpdec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lpdec_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["lpdec_ctx_create", "lpdec_code_create", "lpdec_set_option", "lpdec_decode",
              "lpdec_decode_batch", "lpdec_server_create", "lpdec_server_submit", "lpdec_server_poll",
              "lpdec_server_destroy", "lpdec_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0902_0657_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblpdec.so not built (run __graft_entry__.build())")
    L = _lib.load()
    for n in declared():
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTED) == declared()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_0902_0657_amd import _lib
    with pytest.raises(ImportError):
        _lib._lib = None
        try:
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = None
