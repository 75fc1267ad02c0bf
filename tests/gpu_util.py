"""Helpers shared by the GPU tests: device planes from the seeded generator and
the FP32 score tolerance."""
import numpy as np
import torch

from paper_1504_01883_amd import lbpf, synth


def require_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def stacked_planes(grey: np.ndarray, depth: np.ndarray):
    """[n, h, w] host crops -> one device image (h*n rows) and its boxes."""
    n, h, w = depth.shape
    g, z = lbpf.to_device_planes(grey.reshape(n * h, w), depth.reshape(n * h, w))
    return [(g, z)], synth.stacked_boxes(n, w, h)


def host_planes(grey: np.ndarray, depth: np.ndarray):
    n, h, w = depth.shape
    return [(grey.reshape(n * h, w), depth.reshape(n * h, w))], synth.stacked_boxes(n, w, h)


def ragged_crops(n, n_ident, seed_workload=synth.W_RAGGED, lo=3, hi=300):
    """n crops with independent random sizes in [lo, hi], each its own image."""
    rng = np.random.default_rng([synth.SEED, seed_workload, 424242])
    crops = []
    for i in range(n):
        w, h = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        crops.append(synth.render_crop(w, h, seed_workload, i % n_ident, 2000 + i))
    return crops


def score_tolerance(X, W, b):
    """1e-5 relative to the dot product's condition scale sum_j |W_kj x_j| + |b_k|."""
    scale = np.abs(X.astype(np.float64)) @ np.abs(W.astype(np.float64)).T + \
        np.abs(b.astype(np.float64))[None, :]
    return 1e-5 * scale
