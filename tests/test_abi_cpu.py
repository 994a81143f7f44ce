"""CPU-side checks of the C-ABI library: it loads, exports every function that
include/tsl.h declares, and its host-only entry points behave (no device use)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsl.h")
LIB = os.path.join(ROOT, "paper_1609_04104_amd", "libtsl.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libtsl.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(tsl_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_expected_calls():
    names = declared_functions()
    for must in ("tsl_open", "tsl_push_lines", "tsl_push_points", "tsl_sample_lines", "tsl_step_many",
                 "tsl_close", "tsl_status", "tsl_fft2", "tsl_pool_create", "tsl_open_in_pool"):
        assert must in names


def test_library_exports_every_declared_function():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_lists_every_declared_function():
    from paper_1609_04104_amd import tsl
    assert sorted(tsl.EXPORTS) == declared_functions()


def test_codelets_match_direct_dft_on_host():
    from paper_1609_04104_amd import tsl
    assert tsl.selftest_codelets() < 3e-7


def test_host_queries():
    from paper_1609_04104_amd import tsl
    for n in (8, 64, 120, 128, 160, 192, 200, 256, 320, 384, 512):
        assert tsl.size_supported(n)
    for n in (7, 11, 1000, 0, -4, 1024):
        assert not tsl.size_supported(n)
    fp = tsl.footprint(256, 256, 32)
    assert fp >= 256 * 256 * 8 + 4 * 256 * 32 * 8
    assert tsl.footprint(256, 256, 64) > fp
    with pytest.raises(tsl.TslError) as e:
        tsl.footprint(250, 256, 32)
    assert e.value.code == tsl.EUNSUPPORTED
    with pytest.raises(tsl.TslError) as e:
        tsl.footprint(256, 256, 0)
    assert e.value.code == tsl.EINVAL
    with pytest.raises(tsl.TslError):
        tsl.footprint(256, 256, tsl.MAX_R + 1)


def test_pool_accounting_on_host():
    from paper_1609_04104_amd import tsl
    p = tsl.Pool(1 << 20)
    assert p.used() == (0, 1 << 20)
    p.destroy()


def test_prepared_batch_argument_errors_on_host():
    """The prepared-batch calls reject bad arguments before any device call."""
    from paper_1609_04104_amd import tsl
    L = tsl.lib()
    out = ctypes.c_void_p(1)
    assert L.tsl_batch_create(None, 1, None, 0, ctypes.byref(out)) == tsl.EINVAL
    assert out.value is None                         # *out is cleared on error
    assert L.tsl_batch_create(None, 0, None, 0, ctypes.byref(out)) == tsl.EINVAL
    assert L.tsl_batch_create(None, 1, None, 0, None) == tsl.EINVAL
    hs = (ctypes.c_void_p * 1)(None)
    fs = (tsl.Frame * 1)()
    assert L.tsl_batch_create(hs, 1, fs, 0, ctypes.byref(out)) == tsl.EINVAL     # null sequence
    assert L.tsl_batch_create(hs, 1, fs, 0x80, ctypes.byref(out)) == tsl.EINVAL  # unknown flag
    assert L.tsl_batch_launch(None, None) == tsl.EINVAL
    assert L.tsl_batch_destroy(None) == tsl.OK
