"""The C-ABI library loads and exports every symbol the public header declares."""
import ctypes
import os
import re

import pytest

import paper_2609_05960_amd as gtp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "gtpower.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"\b(gtp_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_header_symbols():
    if not os.path.exists(gtp.SO_PATH):
        gtp.build()
    L = ctypes.CDLL(gtp.SO_PATH)
    syms = header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), f"{s} not exported"
    assert set(syms) == set(gtp.ABI_SYMBOLS)


def test_null_and_no_device_errors():
    L = gtp.load_library()
    assert L.gtp_create(None, 0, None) == 1  # INVALID_ARG
    assert L.gtp_destroy(None) == 0
    assert L.gtp_last_error(None) == b"null context"
    assert L.gtp_sync(None) == 1
    h = ctypes.c_void_p()
    rc = L.gtp_create(ctypes.byref(h), 99, None)  # no such device
    assert rc == 1 and not h.value


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        gtp.load_library(str(tmp_path / "nope.so"))
