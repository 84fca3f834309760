"""The C-ABI library loads and exports every entry point include/mak.h
declares (no device calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mak.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mak_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2110_08868_amd as mak
    if not os.path.exists(mak.LIB_PATH):
        from paper_2110_08868_amd import build
        build.build()
    return mak.load_library()


def test_header_declares_expected_entry_points():
    import paper_2110_08868_amd as mak
    assert declared_symbols() == sorted(mak.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_default_options_and_estimate(lib):
    import paper_2110_08868_amd as mak
    o = mak.default_options()
    assert o["precision"] == 0 and o["max_newton"] > 0 and o["cg_rtol"] > 0
    assert o["grid_occupancy"] > 0
    small = mak.memory_estimate(4096)
    big = mak.memory_estimate(128 ** 3)
    assert 0 < small < big


def test_null_arguments_rejected_without_device(lib):
    # a NULL context is rejected before any device call
    assert lib.mak_laguerre_cells(None, None, None, 0, 1.0, None, None, None, None, None) == 1
    assert lib.mak_solve(None, None, 0, 1.0, 1e-6, None, None, None, None, None) == 1
    out = ctypes.c_void_p()
    # NULL out pointer
    assert lib.mak_create(None, 0, None) == 1


def test_device_bytes_counter_without_device(lib):
    """The library's device-memory counter reads (zero: nothing allocated
    without a device) and its peak resets to the live value."""
    import paper_2110_08868_amd as mak
    live, peak = mak.device_bytes(reset_peak=True)
    assert live == 0 and peak == 0
