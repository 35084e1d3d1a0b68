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


def test_fixed_point_bits():
    """Host-side range check of the bin accumulators: the largest m <= 40 with
    2^m * bound < 2^62 and 2^m * 1e-6 * leak < 2^30, UNSUPPORTED below 30."""
    f = gtp.fixed_point_bits
    # 1M gates at 50 ps bins: the finest unit
    assert f(300, 50, 500.0, 800.0, 800.0) == 40
    for n, D, e, r, lk in ((10 ** 6, 1 << 22, 430.0, 800.0, 800.0), (5 * 10 ** 5, 1 << 22, 430.0, 6.4e-3, 800.0),
                           (1, 1, 1.0, 1.0, 1.0e4)):
        m = f(n, D, e, r, lk)
        bound = n * e + D * r
        assert 30 <= m <= 40
        assert 2.0 ** m * bound < 2.0 ** 62 and 2.0 ** m * 1e-6 * lk < 2.0 ** 30
        if m < 40:   # maximal: one more bit would break a bound
            assert 2.0 ** (m + 1) * bound >= 2.0 ** 62 or 2.0 ** (m + 1) * 1e-6 * lk >= 2.0 ** 30
    with pytest.raises(gtp.GtpError) as ei:
        f(10 ** 9, 1 << 22, 1.0e4, 1.0e4, 800.0)
    assert ei.value.status == "UNSUPPORTED"
    with pytest.raises(gtp.GtpError) as ei:
        f(-1, 50, 1.0, 1.0, 1.0)
    assert ei.value.status == "INVALID_ARG"


def test_expand_when_golden():
    """The hand-computed state-pattern fixture through the host expansion."""
    import json
    with open(os.path.join(ROOT, "tests", "golden", "when_patterns.json")) as f:
        fx = json.load(f)
    out = gtp.expand_when(fx["n_pins"], fx["care"], fx["value"], [10, 11, 12], -5)
    assert out.tolist() == [[10, 11, 12][k] for k in fx["expect_first_match"]]
    p = fx["partial"]
    out = gtp.expand_when(fx["n_pins"], p["care"], p["value"], [10, 11], -5)
    assert out.tolist() == [-5 if k < 0 else [10, 11][k] for k in p["expect_first_match"]]


@pytest.mark.parametrize("n_pins", [0, 1, 5, 9, 16])
def test_expand_when_matches_pattern_scan(n_pins):
    """Every entry of the expansion equals the item of the oracle's
    first-match scan over the patterns (default where none matches)."""
    import numpy as np

    import oracle
    O = oracle.get()
    rng = np.random.default_rng(n_pins)
    for trial in range(3):
        n_pat = int(rng.integers(0, 12))
        care = np.zeros(n_pat, np.uint32)
        for k in range(n_pat):
            for p in range(n_pins):
                if rng.random() < min(0.5, 3.0 / max(n_pins, 1)):
                    care[k] |= np.uint32(1 << p)
        value = rng.integers(0, 1 << 32, n_pat, dtype=np.uint64).astype(np.uint32)
        item = rng.integers(-100, 100, n_pat).astype(np.int32)
        out = gtp.expand_when(n_pins, care, value, item, 7777)
        states = range(1 << n_pins) if n_pins <= 9 else rng.integers(0, 1 << n_pins, 3000)
        for s in states:
            k = O.pattern_scan(care, value, int(s))
            assert out[s] == (7777 if k < 0 else item[k]), (n_pins, trial, int(s))


def test_expand_when_errors():
    L = gtp.load_library()
    import numpy as np
    out = np.zeros(1 << 4, np.int32)
    care = np.array([1 << 4], np.uint32)   # a pin above n_pins
    z = np.zeros(1, np.uint32)
    it = np.zeros(1, np.int32)
    assert L.gtp_expand_when(4, 1, care.ctypes.data, z.ctypes.data, it.ctypes.data, 0, out.ctypes.data) == 1
    assert L.gtp_expand_when(17, 0, None, None, None, 0, out.ctypes.data) == 1
    assert L.gtp_expand_when(4, 1, None, None, None, 0, out.ctypes.data) == 1
    assert L.gtp_expand_when(4, 0, None, None, None, 3, out.ctypes.data) == 0
    assert out.tolist() == [3] * 16
