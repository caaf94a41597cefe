"""The C ABI boundary, checked without a GPU: the library loads, exports every
entry point declared in include/rgs.h, and rejects invalid arguments before
touching a device."""

import ctypes
import os
import re

import pytest

import paper_2011_05090_amd as rgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rgs_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rgs.LIB_PATH):
        pytest.fail("librgs.so is not built (python -m paper_2011_05090_amd.build)")
    return rgs.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("rgs_qr", "rgs_gmres", "rgs_create", "rgs_destroy", "rgs_sketch_apply",
                 "rgs_sketch_materialize", "rgs_stencil_apply", "rgs_status_string", "rgs_abi_version"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    assert set(declared_functions()) == set(rgs.SIGNATURES)


def test_abi_version_and_status_strings(lib):
    assert rgs.rgs_abi_version() == 7
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = rgs.status_string(code)
        assert s and "unknown" not in s
    assert "unknown" in rgs.status_string(-99)


def test_null_arguments_are_rejected_without_a_device(lib):
    assert lib.rgs_create(None, 0, None) == rgs.RGS_EINVAL
    d = rgs.qr_desc(1000, 10, 64)
    assert lib.rgs_qr(None, ctypes.byref(d), None, 1000, None, 1000, None, 10, None, 64, None) == rgs.RGS_EINVAL
    assert lib.rgs_qr_noalloc(None, ctypes.byref(d), None, 1000, None, 1000, None, 10, None, 64,
                              None) == rgs.RGS_EINVAL
    assert lib.rgs_destroy(None) == rgs.RGS_EINVAL
    A = rgs.stencil7((4, 4, 4), (6, -1, -1, -1, -1, -1, -1))
    g = rgs.gmres_desc(10, 40, 1e-6)
    assert lib.rgs_gmres(None, ctypes.byref(A), ctypes.byref(g), None, None, None, 0, None) == rgs.RGS_EINVAL
    assert lib.rgs_stencil_apply(None, ctypes.byref(A), 1, None, None) == rgs.RGS_EINVAL


def test_struct_layouts_match_header_sizes():
    # field-by-field layout of the ABI structs (x86-64, natural alignment)
    assert ctypes.sizeof(rgs.QrDesc) == 8 * 4 + 4 * 6
    assert ctypes.sizeof(rgs.Stencil7) == 8 * 3 + 8 * 7
    assert ctypes.sizeof(rgs.GmresDesc) == 8 * 5 + 4 * 5 + 4   # padded to a multiple of 8
    assert ctypes.sizeof(rgs.Report) == 8 * 14
    assert ctypes.sizeof(rgs.QrItem) == 8 * 11
    assert ctypes.sizeof(rgs.GmresItem) == ctypes.sizeof(rgs.Stencil7) + 8 * 4


def test_omega_bar_helper_matches_the_oracle(lib):
    """rgs_omega_bar is a host function: Prop. 3.7's formula, checked against
    the oracle's, both branches of the maximum, and NaN propagation."""
    import math
    from oracle import metrics
    for smin, smax, eps in ((0.9, 1.05, 0.05), (0.99, 1.2, 0.25), (1.0, 1.0, 0.0), (0.5, 0.6, 0.1)):
        assert rgs.rgs_omega_bar(smin, smax, eps) == pytest.approx(metrics.omega_bar_from(smin, smax, eps),
                                                                   rel=1e-15, abs=1e-15)
    assert math.isnan(rgs.rgs_omega_bar(float("nan"), 1.0, 0.05))
    assert math.isnan(rgs.rgs_omega_bar(1.0, float("nan"), 0.05))
