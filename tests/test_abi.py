"""CPU-side checks of the C ABI: the library builds, loads, and exports every
entry point include/lbpf.h declares. No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbpf.h")
LIB = os.path.join(ROOT, "paper_1504_01883_amd", "liblbpf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbpf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1504_01883_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("lbpf_create", "lbpf_destroy", "lbpf_feature_dim", "lbpf_features",
                 "lbpf_weights_create", "lbpf_weights_destroy", "lbpf_score",
                 "lbpf_debug_codes", "lbpf_status_string", "lbpf_last_error"):
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_1504_01883_amd import lbpf
    assert sorted(lbpf.EXPORTS) == declared_functions()


def test_status_strings_and_version(lib):
    lib.lbpf_status_string.restype = ctypes.c_char_p
    lib.lbpf_status_string.argtypes = [ctypes.c_int]
    names = [lib.lbpf_status_string(s).decode() for s in (0, -1, -2, -3, -4)]
    assert names == ["LBPF_OK", "LBPF_E_INVALID", "LBPF_E_BUDGET", "LBPF_E_HIP",
                     "LBPF_E_UNSUPPORTED"]
    lib.lbpf_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.lbpf_version()
    lib.lbpf_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.lbpf_last_error(), bytes)


def test_null_arguments_rejected_without_device_work(lib):
    """Argument checks run before any HIP call: NULL handles fail cleanly."""
    lib.lbpf_feature_dim.restype = ctypes.c_int32
    lib.lbpf_feature_dim.argtypes = [ctypes.c_void_p]
    assert lib.lbpf_feature_dim(None) == -1
    lib.lbpf_features.restype = ctypes.c_int
    lib.lbpf_features.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int32, ctypes.c_void_p,
                                                          ctypes.c_int32] + [ctypes.c_void_p] * 3
    assert lib.lbpf_features(None, None, 0, None, 0, None, None, None) == -1
    lib.lbpf_score.restype = ctypes.c_int
    lib.lbpf_score.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32] + \
        [ctypes.c_void_p] * 4
    assert lib.lbpf_score(None, None, 0, None, None, None, None) == -1
    lib.lbpf_create.restype = ctypes.c_int
    lib.lbpf_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    assert lib.lbpf_create(None, None, 0) == -1


def test_warp_crop_bytes(lib):
    lib.lbpf_warp_crop_bytes.restype = ctypes.c_size_t
    lib.lbpf_warp_crop_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    for w, h in [(3, 3), (200, 200), (255, 97), (1024, 1024)]:
        b = lib.lbpf_warp_crop_bytes(w, h)
        assert b % 256 == 0
        assert b >= 3 * w * h + 3 * 7  # both planes plus the row over-read slack
    for w, h in [(2, 5), (5, 2), (1025, 5), (5, 1025), (-1, 5)]:
        assert lib.lbpf_warp_crop_bytes(w, h) == 0
    lib.lbpf_features_warped.restype = ctypes.c_int
    lib.lbpf_features_warped.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]
    assert lib.lbpf_features_warped(None, None, 0, None, 0, None, 0, None, None, None) == -1


@pytest.mark.parametrize("w", [48, 97, 128, 199, 200, 201, 256, 640])
def test_resize_frame_samples_stay_in_the_box(w):
    """Host helper: the corner samples of a resize frame land on the box's
    first and last pixel in both axes (by linearity, every sample is inside)."""
    from paper_1504_01883_amd import lbpf
    x0, y0, h = 13, 7, int(w * 1.1)
    for out in (200, 64, 3, 1024):
        ux, uy, vx, vy, tx, ty = lbpf.resize_frame(x0, y0, w, h, out, out)
        sx = lambda x: (ux * x + tx) >> 16
        sy = lambda y: (vy * y + ty) >> 16
        assert uy == 0 and vx == 0
        assert x0 <= sx(0) and sx(out - 1) <= x0 + w - 1
        assert y0 <= sy(0) and sy(out - 1) <= y0 + h - 1
        if out == w:
            assert [sx(x) for x in range(out)] == list(range(x0, x0 + w))
