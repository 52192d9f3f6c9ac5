"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/gs3.h declares, and its host-only entry points
(constants, status strings, workspace sizing, argument validation) behave."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs3.h")
LIB = os.path.join(ROOT, "paper_2410_11419_amd", "libgs3.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs3_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["gs3_preprocess", "gs3_shadow_splat", "gs3_render", "gs3_project", "gs3_bin"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libgs3.so not built: python -m paper_2410_11419_amd.build"
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_2410_11419_amd import gs3
    assert set(declared_functions()) == set(gs3.EXPORTED)


def test_host_only_entry_points():
    from paper_2410_11419_amd import gs3
    k = gs3.default_consts()
    assert k.cutoff == pytest.approx(4.5) and k.shadow_bias == pytest.approx(0.015)
    assert k.alpha_min == pytest.approx(1 / 255) and k.alpha_max == pytest.approx(0.99)
    assert k.t_min == pytest.approx(1e-4) and k.dilation == pytest.approx(0.3)
    assert k.near_plane == pytest.approx(0.2) and k.clamp_frac == pytest.approx(1.3)
    assert gs3._lib.gs3_status_string(-3) == b"GS3_PAIR_CAPACITY_EXCEEDED"
    size = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(1000, 128, 96, 50000, C.byref(size)) == 0
    assert size.value > 50000 * 16
    big = C.c_size_t()
    assert gs3._lib.gs3_view_workspace_size(1000, 128, 96, 100000, C.byref(big)) == 0
    assert big.value > size.value
    assert gs3._lib.gs3_view_workspace_size(-1, 128, 96, 10, C.byref(size)) == gs3.GS3_INVALID_ARG
    assert gs3._lib.gs3_view_workspace_size(10, 0, 96, 10, C.byref(size)) == gs3.GS3_INVALID_ARG
    assert b"invalid" in gs3._lib.gs3_last_error()
    # a NULL view buffer is rejected before any device work
    assert gs3._lib.gs3_view_pair_count(None, None, None) == gs3.GS3_INVALID_ARG
    vb = gs3.gs3_viewbuf(C.c_void_p(256), 10, 100, 64, 64, 1000)   # too small a workspace
    n = C.c_int64()
    assert gs3._lib.gs3_view_pair_count(C.byref(vb), C.byref(n), None) == gs3.GS3_WORKSPACE_TOO_SMALL
    vb = gs3.gs3_viewbuf(C.c_void_p(257), 1 << 30, 100, 64, 64, 1000)  # misaligned
    assert gs3._lib.gs3_view_pair_count(C.byref(vb), C.byref(n), None) == gs3.GS3_INVALID_ARG
