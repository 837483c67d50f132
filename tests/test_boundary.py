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


def test_argument_errors_are_reported_before_any_device_work():
    """Null handles and invalid devices come back as LPDEC_EINVAL / LPDEC_EDEVICE from the C ABI
    itself (runs on a host without a GPU: these paths check their arguments first)."""
    import ctypes as C
    from paper_0902_0657_amd import _lib
    L = _lib.load()
    p = C.c_void_p()
    assert L.lpdec_ctx_create(0, None) == _lib.EINVAL
    assert L.lpdec_ctx_create(-1, C.byref(p)) == _lib.EDEVICE and not p.value
    assert L.lpdec_ctx_destroy(None) == _lib.EINVAL
    assert L.lpdec_set_option(None, _lib.OPT["PRECISION"], 1.0) == _lib.EINVAL
    v = C.c_double()
    assert L.lpdec_get_option(None, _lib.OPT["PRECISION"], C.byref(v)) == _lib.EINVAL
    assert L.lpdec_code_destroy(None) == _lib.EINVAL
    assert L.lpdec_decode_batch(None, None, 1, None, 0, None, None, None, None, None, None) == _lib.EINVAL
    assert L.lpdec_server_poll(None, 0, None, None, None, None) == _lib.EINVAL
    assert L.lpdec_server_destroy(None) == _lib.EINVAL
    assert L.lpdec_last_error(None) == b"null context"
