"""CPU oracle for the depth-fused LBP face-recognition path (arXiv 1504.01883).

TEST INFRASTRUCTURE. The plain, slow reference that the GPU library is checked
against. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product path (the HIP library and its
binding) never does. It shares no code with the GPU path.

The arithmetic lives in ``lbpf_ref.c`` (plain C loops, built with gcc); this
module only marshals numpy arrays into it. Each wrapper names the passage of
the paper it follows:

* ``median``     -- depth region of interest (abstract and Sec. 1: depth
                    reduces cost and removes pose effects); reading: lower
                    median of the crop's non-zero depth.
* ``lbp_code_*`` -- Sec. 2.4, Eq. 2, Fig. 7.
* ``uniform_bin``-- uniform patterns of the LBP operator of ref. [16].
* ``features``   -- Sec. 2.4, Eq. 3 (regional histograms); Sec. 3 (grey u8 and
                    ushort depth).
* ``features_warped`` -- Sec. 2.1, Eq. 1 (affine frame p' = x u + y v + t)
                    and Sec. 3 (faces resized to 200 x 200): nearest samples
                    through a 16.16 fixed-point frame, then ``features``.
* ``track``      -- Sec. 2.3, Fig. 4 (nearest box centre in the next frame).
* ``score_f64``  -- Sec. 2.5 (one hyperplane per person; largest score wins).
* ``train_ovr_f64`` -- Sec. 2.5 (max-margin, one person vs the rest).

Parity unpinned: the neighbour order of the LBP code (the paper's figure is
lost); the SVM hyper-parameters (C, bias handling, feature scaling). Both are
documented readings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "lbpf_ref.c"
_LIB = _HERE / "liblbpf_ref.so"

MAP_U59, MAP_FULL256 = 0, 1
MOD_BOTH, MOD_GREY, MOD_DEPTH = 0, 1, 2


def build(force: bool = True) -> Path:
    """Compile lbpf_ref.c into liblbpf_ref.so with gcc (-O2, no fast-math)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-o", str(tmp), str(_SRC), "-lpthread", "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Image(ctypes.Structure):
    _fields_ = [("grey", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("grey_pitch", ctypes.c_int32), ("depth_pitch", ctypes.c_int32)]


class _Box(ctypes.Structure):
    _fields_ = [("image", ctypes.c_int32), ("x", ctypes.c_int32), ("y", ctypes.c_int32),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32)]


class _Frame(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("ux", "uy", "vx", "vy", "tx", "ty")]


class _WarpBox(ctypes.Structure):
    _fields_ = [("image", ctypes.c_int32), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("grey", _Frame), ("depth", _Frame)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = ctypes.CDLL(str(_LIB))
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.lbpf_ref_median.restype = i32
        lib.lbpf_ref_median.argtypes = [vp, i32, i32, i32]
        lib.lbpf_ref_lbp_code_u8.restype = i32
        lib.lbpf_ref_lbp_code_u8.argtypes = [vp, i32, i32, i32]
        lib.lbpf_ref_lbp_code_u16.restype = i32
        lib.lbpf_ref_lbp_code_u16.argtypes = [vp, i32, i32, i32]
        lib.lbpf_ref_is_uniform.restype = i32
        lib.lbpf_ref_is_uniform.argtypes = [i32]
        lib.lbpf_ref_uniform_bin.restype = i32
        lib.lbpf_ref_uniform_bin.argtypes = [i32]
        lib.lbpf_ref_feature_dim.restype = i32
        lib.lbpf_ref_feature_dim.argtypes = [i32, i32, i32, i32]
        lib.lbpf_ref_codes.restype = None
        lib.lbpf_ref_codes.argtypes = [vp, i32, vp, i32, i32, i32, i32, vp, vp, vp]
        lib.lbpf_ref_features.restype = i32
        lib.lbpf_ref_features.argtypes = [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, i32]
        lib.lbpf_ref_features_warped.restype = i32
        lib.lbpf_ref_features_warped.argtypes = [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp,
                                                 vp, vp, i32]
        lib.lbpf_ref_track.restype = None
        lib.lbpf_ref_track.argtypes = [vp, vp, i32, vp, vp, i32, i64, vp, vp]
        lib.lbpf_ref_score_f64.restype = None
        lib.lbpf_ref_score_f64.argtypes = [vp, i64, vp, vp, i32, i32, vp, vp, i32]
        lib.lbpf_ref_train_ovr_f64.restype = i32
        lib.lbpf_ref_train_ovr_f64.argtypes = [vp, vp, i32, i32, i32, ctypes.c_double,
                                               ctypes.c_double, i32, ctypes.c_uint64, vp, vp, i32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def median(depth: np.ndarray) -> int:
    """Lower median of the non-zero values of a 2-D u16 crop, or -1 if none."""
    z = _c(depth, np.uint16)
    h, w = z.shape
    return int(_load().lbpf_ref_median(_ptr(z), w, w, h))


def lbp_code_u8(img: np.ndarray, y: int, x: int) -> int:
    a = _c(img, np.uint8)
    return int(_load().lbpf_ref_lbp_code_u8(_ptr(a), a.shape[1], y, x))


def lbp_code_u16(img: np.ndarray, y: int, x: int) -> int:
    a = _c(img, np.uint16)
    return int(_load().lbpf_ref_lbp_code_u16(_ptr(a), a.shape[1], y, x))


def is_uniform(code: int) -> bool:
    return bool(_load().lbpf_ref_is_uniform(code))


def uniform_bin(code: int) -> int:
    return int(_load().lbpf_ref_uniform_bin(code))


def feature_dim(grid_x=8, grid_y=8, mapping=MAP_U59, modality=MOD_BOTH) -> int:
    return int(_load().lbpf_ref_feature_dim(grid_x, grid_y, mapping, modality))


def codes(grey: np.ndarray, depth: np.ndarray, window: int = 150):
    """Per-pixel (grey code, depth code, mask) of one crop; border entries 0."""
    g = _c(grey, np.uint8)
    z = _c(depth, np.uint16)
    h, w = z.shape
    assert g.shape == (h, w)
    gc = np.zeros((h, w), np.uint8)
    zc = np.zeros((h, w), np.uint8)
    mk = np.zeros((h, w), np.uint8)
    _load().lbpf_ref_codes(_ptr(g), w, _ptr(z), w, w, h, window, _ptr(gc), _ptr(zc), _ptr(mk))
    return gc, zc, mk


def features(images, boxes, grid_x=8, grid_y=8, mapping=MAP_U59, window=150,
             modality=MOD_BOTH, n_threads=1):
    """Features of every box.

    images: list of (grey u8 [H,W] or None, depth u16 [H,W]) host arrays.
    boxes:  int array [n, 5] of (image, x, y, w, h).
    Returns (feat f32 [n, D], counts u32 [n, D], n_in i64 [n]).
    """
    lib = _load()
    keep = []
    imgs = (_Image * max(1, len(images)))()
    for i, (g, z) in enumerate(images):
        z = _c(z, np.uint16)
        g = _c(g if g is not None else np.zeros_like(z, dtype=np.uint8), np.uint8)
        keep += [g, z]
        imgs[i] = _Image(_ptr(g), _ptr(z), z.shape[1], z.shape[0], g.shape[1], z.shape[1])
    bx = _c(np.asarray(boxes, np.int32).reshape(-1, 5), np.int32)
    n = bx.shape[0]
    D = feature_dim(grid_x, grid_y, mapping, modality)
    feat = np.zeros((n, D), np.float32)
    counts = np.zeros((n, D), np.uint32)
    n_in = np.zeros((n,), np.int64)
    rc = lib.lbpf_ref_features(ctypes.addressof(imgs), len(images), _ptr(bx), n, grid_x, grid_y,
                               mapping, window, modality, _ptr(counts), _ptr(feat), _ptr(n_in),
                               n_threads)
    if rc != 0:
        raise ValueError("oracle: invalid feature arguments (box outside image, side < 3, ...)")
    return feat, counts, n_in


def _images(images, keep):
    imgs = (_Image * max(1, len(images)))()
    for i, (g, z) in enumerate(images):
        z = _c(z, np.uint16)
        g = _c(g if g is not None else np.zeros_like(z, dtype=np.uint8), np.uint8)
        keep += [g, z]
        imgs[i] = _Image(_ptr(g), _ptr(z), z.shape[1], z.shape[0], g.shape[1], z.shape[1])
    return imgs


def features_warped(images, boxes, grid_x=8, grid_y=8, mapping=MAP_U59, window=150,
                    modality=MOD_BOTH):
    """Features of warped crops.

    boxes: sequence of (image, w, h, grey_frame, depth_frame) with each frame a
    6-tuple (ux, uy, vx, vy, tx, ty) in 16.16 fixed point: crop pixel (x, y)
    samples source (floor((ux x + vx y + tx) / 2^16), floor((uy x + vy y + ty) / 2^16)).
    Returns (feat f32 [n, D], counts u32 [n, D], n_in i64 [n])."""
    lib = _load()
    keep = []
    imgs = _images(images, keep)
    n = len(boxes)
    bx = (_WarpBox * max(1, n))()
    for i, (im, w, h, gf, zf) in enumerate(boxes):
        bx[i] = _WarpBox(im, w, h, _Frame(*[int(v) for v in gf]), _Frame(*[int(v) for v in zf]))
    D = feature_dim(grid_x, grid_y, mapping, modality)
    feat = np.zeros((n, D), np.float32)
    counts = np.zeros((n, D), np.uint32)
    n_in = np.zeros((n,), np.int64)
    rc = lib.lbpf_ref_features_warped(ctypes.addressof(imgs), len(images), ctypes.addressof(bx),
                                      n, grid_x, grid_y, mapping, window, modality, _ptr(counts),
                                      _ptr(feat), _ptr(n_in), 1)
    if rc != 0:
        raise ValueError("oracle: invalid warped-feature arguments (sample outside the plane, ...)")
    return feat, counts, n_in


def crop_features(grey: np.ndarray, depth: np.ndarray, **kw):
    """Features of a single whole crop (convenience)."""
    h, w = np.asarray(depth).shape
    f, c, n = features([(grey, depth)], [[0, 0, 0, w, h]], **kw)
    return f[0], c[0], int(n[0])


def track(prev_boxes, prev_stream, cur_boxes, cur_stream, gate2=0):
    """Nearest-centre association of previous-frame tracks to current boxes.
    Boxes are [n, 4] (x, y, w, h); streams [n]. Returns (match [P], owner [C])."""
    pb = _c(np.asarray(prev_boxes).reshape(-1, 4), np.int32)
    ps = _c(prev_stream, np.int32)
    cb = _c(np.asarray(cur_boxes).reshape(-1, 4), np.int32)
    cs = _c(cur_stream, np.int32)
    P, C = pb.shape[0], cb.shape[0]
    assert ps.shape == (P,) and cs.shape == (C,)
    match = np.zeros(P, np.int32)
    owner = np.zeros(C, np.int32)
    _load().lbpf_ref_track(_ptr(pb), _ptr(ps), P, _ptr(cb), _ptr(cs), C, int(gate2),
                           _ptr(match), _ptr(owner))
    return match, owner


def score_f64(X: np.ndarray, W: np.ndarray, b: np.ndarray, want_scores=True, n_threads=1):
    """S = X W^T + b in double (j ascending) and argmax (lowest index on ties)."""
    X = _c(X, np.float32)
    W = _c(W, np.float32)
    b = _c(b, np.float32)
    N, D = X.shape
    K = W.shape[0]
    assert W.shape == (K, D) and b.shape == (K,)
    S = np.zeros((N, K), np.float64) if want_scores else None
    am = np.zeros((N,), np.int32)
    _load().lbpf_ref_score_f64(_ptr(X), N, _ptr(W), _ptr(b), K, D,
                               _ptr(S) if S is not None else None, _ptr(am), n_threads)
    return S, am


def train_ovr_f64(X: np.ndarray, labels: np.ndarray, K: int, C: float = 1.0, eps: float = 1e-6,
                  max_epochs: int = 200, seed: int = 150401883, n_threads: int = 1):
    """One-vs-rest linear SVM (dual coordinate descent) in double.

    Returns (W f64 [K, D], b f64 [K], epochs used by the slowest class).
    """
    X = _c(X, np.float32)
    y = _c(labels, np.int32)
    N, D = X.shape
    W = np.zeros((K, D), np.float64)
    b = np.zeros((K,), np.float64)
    ep = _load().lbpf_ref_train_ovr_f64(_ptr(X), _ptr(y), N, D, K, C, eps, max_epochs, seed,
                                        _ptr(W), _ptr(b), n_threads)
    return W, b, int(ep)
